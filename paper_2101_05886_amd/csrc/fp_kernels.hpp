// fp_kernels.hpp -- gfx950 kernels of the free-stream-preserving residual:
// direction sweeps, cell-face flux evaluation, metrics, CFL and state checks.
// Instantiated by the fp_inst_*.hip translation units and launched by fp_api.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fp_device.hpp"

namespace fpk {

// Geometry of one structured block as the kernels see it.  Offsets are in
// elements of one variable array; `base` is the offset of interior node
// (0,0,0); sd[d] is the stride of axis d.
struct GeoK {
    int n[3];
    int g;
    int bc[3];
    long sd[3];
    long vol;
    long base;
};

// What a sweep does with the flux difference d = F'_{i+1/2} - F'_{i-1/2} of
// its direction at node `off`:
//   FIRST: R = -d        MID: R = R - d
//   LAST_RES: out = (R - d) / (1/J)
//   LAST_RK:  k = (R - d) / (1/J); u = qin + dt k;
//             out = u (first stage) or a qn + b u (TVD RK3 stages 2, 3)
enum { EPI_FIRST = 0, EPI_MID = 1, EPI_LAST_RES = 2, EPI_LAST_RK = 3 };

struct EpiK {
    int mode;
    int stage0;
    double* R;
    double* out;
    const double* metV;
    const double* qin;
    const double* qn;
    double dt, a, b;
};

template <int NV>
__device__ __forceinline__ void epilogue(const EpiK& ep, long vol, long off, const double (&d)[NV]) {
    if (ep.mode == EPI_FIRST) {
#pragma unroll
        for (int v = 0; v < NV; ++v) ep.R[v * vol + off] = -d[v];
    } else if (ep.mode == EPI_MID) {
#pragma unroll
        for (int v = 0; v < NV; ++v) ep.R[v * vol + off] -= d[v];
    } else if (ep.mode == EPI_LAST_RES) {
        const double V = ep.metV[off];
#pragma unroll
        for (int v = 0; v < NV; ++v) ep.out[v * vol + off] = (ep.R[v * vol + off] - d[v]) / V;
    } else {
        const double V = ep.metV[off];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const long o = v * vol + off;
            const double k = (ep.R[o] - d[v]) / V;
            const double u = ep.qin[o] + ep.dt * k;
            ep.out[o] = ep.stage0 ? u : ep.a * ep.qn[o] + ep.b * u;
        }
    }
}

// Load the stencil of face i+1/2 of the line starting at offset lb (node 0 of
// the line) along axis DIR.  State values outside the interior come from the
// periodic image of qs or, on a frozen axis, from the ghost layers of qb.
// Metrics are read directly (their ghost layers are filled by fp_metrics).
template <int DIM, int DIR, int Y>
__device__ __forceinline__ void load_stencil(const GeoK& G, const double* __restrict__ met,
                                             const double* qs, const double* qb, long lb, int i,
                                             Stencil<DIM>& st) {
    constexpr int NV = DIM + 2;
    constexpr int NMET = DIM == 3 ? 10 : 5;
    constexpr int r0 = Y == 8 ? 0 : 1;
    constexpr int r1 = Y == 8 ? 8 : 7;
    const long sd = G.sd[DIR];
    const int nd = G.n[DIR];
    const bool per = G.bc[DIR] == 0;
#pragma unroll
    for (int r = r0; r < r1; ++r) {
        const int t = i - 3 + r;
        int tt = t;
        const double* src = qs;
        if (t < 0 || t >= nd) {
            if (per)
                tt = t < 0 ? t + nd : t - nd;
            else
                src = qb;
        }
        const long off = lb + (long)tt * sd;
#pragma unroll
        for (int v = 0; v < NV; ++v) st.q[r][v] = src[v * G.vol + off];
        const long moff = lb + (long)t * sd;
        st.V[r] = met[(NMET - 1) * G.vol + moff];
#pragma unroll
        for (int c = 0; c < DIM; ++c) st.s[r][c] = met[(DIR * DIM + c) * G.vol + moff];
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        if (r >= r0 && r < r1) continue;
#pragma unroll
        for (int v = 0; v < NV; ++v) st.q[r][v] = 0.0;
        st.V[r] = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) st.s[r][c] = 0.0;
    }
}

template <int PREC>
using char_t = typename std::conditional<PREC == 1, float, double>::type;

// xi sweep: 64 lanes evaluate 64 consecutive faces of the flattened face index
// (faces of consecutive xi-lines one after another); waves overlap by one face
// so that every lane but the first takes its left neighbour's flux by a lane
// shift and forms the flux difference of its node.
template <int DIM, int RECON, int Y, int PREC>
__global__ __launch_bounds__(256) void k_sweep_x(GeoK G, SchemeK sk, const double* __restrict__ met,
                                                  const double* qs, const double* qb, EpiK ep) {
    constexpr int NV = DIM + 2;
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const long F = wave * 63 + lane;
    const int nf = G.n[0] + 1;
    const long total = (long)nf * G.n[1] * G.n[2];
    const bool active = F < total;
    double fl[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) fl[v] = 0.0;
    long lb = 0;
    int f = 0;
    if (active) {
        const long line = F / nf;
        f = (int)(F - line * nf);
        const int j = (int)(line % G.n[1]);
        const int k = (int)(line / G.n[1]);
        lb = G.base + (long)j * G.sd[1] + (long)k * G.sd[2];
        Stencil<DIM> st;
        load_stencil<DIM, 0, Y>(G, met, qs, qb, lb, f - 1, st);
        face_flux<DIM, RECON, Y, char_t<PREC>>(st, sk, fl);
    }
    double d[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v] = fl[v] - __shfl_up(fl[v], 1, 64);
    if (active && lane > 0 && f > 0) epilogue<NV>(ep, G.vol, lb + (f - 1), d);
}

// eta / zeta sweeps: one lane per line segment, lanes along i (coalesced);
// each lane marches along the sweep axis and carries the previous face flux.
template <int DIM, int DIR, int RECON, int Y, int PREC>
__global__ __launch_bounds__(256) void k_sweep_march(GeoK G, SchemeK sk,
                                                      const double* __restrict__ met,
                                                      const double* qs, const double* qb, EpiK ep,
                                                      int S, int nseg) {
    constexpr int NV = DIM + 2;
    constexpr int OTH = DIR == 1 ? 2 : 1;
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n0 = G.n[0];
    const int no = G.n[OTH];
    if (tid >= (long)n0 * no * nseg) return;
    const int i = (int)(tid % n0);
    const long rest = tid / n0;
    const int o = (int)(rest % no);
    const int seg = (int)(rest / no);
    const int nd = G.n[DIR];
    const int t0 = seg * S;
    const int t1 = min(t0 + S, nd);
    if (t0 >= t1) return;
    const long lb = G.base + i + (long)o * G.sd[OTH];
    double Fp[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fp[v] = 0.0;
    for (int t = t0 - 1; t < t1; ++t) {
        Stencil<DIM> st;
        load_stencil<DIM, DIR, Y>(G, met, qs, qb, lb, t, st);
        double Fc[NV];
        face_flux<DIM, RECON, Y, char_t<PREC>>(st, sk, Fc);
        if (t >= t0) {
            double d[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) d[v] = Fc[v] - Fp[v];
            epilogue<NV>(ep, G.vol, lb + (long)t * G.sd[DIR], d);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) Fp[v] = Fc[v];
    }
}

// Every face of direction DIR, one lane per face (parity checks).
template <int DIM, int DIR, int RECON, int Y, int PREC>
__global__ __launch_bounds__(256) void k_face_flux(GeoK G, SchemeK sk, const double* __restrict__ met,
                                                    const double* q, double* out) {
    constexpr int NV = DIM + 2;
    int ext[3] = {G.n[0], G.n[1], G.n[2]};
    ext[DIR] += 1;
    const long total = (long)ext[0] * ext[1] * ext[2];
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= total) return;
    int c[3];
    c[0] = (int)(tid % ext[0]);
    c[1] = (int)((tid / ext[0]) % ext[1]);
    c[2] = (int)(tid / ((long)ext[0] * ext[1]));
    long lb = G.base;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (d != DIR) lb += (long)c[d] * G.sd[d];
    Stencil<DIM> st;
    load_stencil<DIM, DIR, Y>(G, met, q, q, lb, c[DIR] - 1, st);
    double fl[NV];
    face_flux<DIM, RECON, Y, char_t<PREC>>(st, sk, fl);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * total + tid] = fl[v];
}

// ---------------------------------------------------------------------------
// launch helpers (defined in the instantiation units)
// ---------------------------------------------------------------------------

struct SweepArgs {
    GeoK G;
    SchemeK sk;
    const double* met;
    const double* qs;
    const double* qb;
    EpiK ep_first, ep_mid, ep_last;
    int S[3];
    int nseg[3];
};

// one full residual evaluation (all sweeps) of the given instantiation
using stage_fn = hipError_t (*)(const SweepArgs&, hipStream_t);
using faceflux_fn = hipError_t (*)(const GeoK&, const SchemeK&, const double*, const double*,
                                   double*, hipStream_t);
// one direction sweep of the given instantiation with epilogue `ep`
using dir_fn = hipError_t (*)(const SweepArgs&, int dir, const EpiK& ep, hipStream_t);

stage_fn get_stage_fn(int ndim, int recon, int Y, int prec);
faceflux_fn get_faceflux_fn(int ndim, int dir, int recon, int Y, int prec);
dir_fn get_dir_fn(int ndim, int recon, int Y, int prec);

}  // namespace fpk
