// fp_kernels.hpp -- gfx950 kernels of the free-stream-preserving residual:
// direction sweeps, cell-face flux evaluation, metrics, CFL and state checks.
// Instantiated by the fp_inst_*.hip translation units and launched by fp_api.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fp_device.hpp"

// Occupancy target of the face kernels: two waves per SIMD fits the FP64
// WENO face (the 6-node x 5-field characteristic values dominate) without
// spilling.  The FP32-mixed xi sweeps of the six-point stencils (WENO5,
// LU5, WENOCU6 with metrics of order up to 6) and the FP64 LU5 ones fit
// three (at most 168 registers) and run at three: their LDS window buffers
// allow it, the eta/zeta rings (72 KB per workgroup) do not; WENO7 and
// eighth-order metrics would spill at three.
#ifndef FP_SWEEP_ATTR
#define FP_SWEEP_ATTR __attribute__((amdgpu_waves_per_eu(2, 2)))
#endif
#define FP_XWAVES(PREC, RECON, Y) \
    ((((PREC) == 1 && (RECON) != 2) || ((PREC) == 0 && (RECON) == 1)) && (Y) != 8 ? 3 : 2)
#define FP_XSWEEP_ATTR(PREC, RECON, Y) \
    __attribute__((amdgpu_waves_per_eu(FP_XWAVES(PREC, RECON, Y), FP_XWAVES(PREC, RECON, Y))))

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

// The eta / zeta sweeps, which apply the final epilogues, take qin and 1/J
// from the stencil rows they staged: qin must be the array the sweep reads
// and metV the metric array's 1/J component.
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

// Global-memory view of a pointer the compiler cannot prove global (one read
// from a table in device memory, as the batched kernels' arrays are):
// accesses through it are global_* instructions, counted only in vmcnt,
// instead of flat_* ones, which also count in lgkmcnt and so hold up every
// wait for LDS reads that follows them.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ gdouble* gmem(double* p) { return (gdouble*)p; }
__device__ __forceinline__ const gdouble* gmem(const double* p) { return (const gdouble*)p; }

// Buffer access to one variable array: the resource (base, size) is
// wave-uniform and lives in scalar registers, every lane supplies a 32-bit
// byte offset, so no 64-bit vector address arithmetic is spent per access.
// Reads past `elems` return 0 by the hardware's range check.  A variable array must stay below 4 GiB (checked
// by the host: at most 2^29 nodes per block, ghosts included).
#define FP_BUF_FLAGS 0x00020000
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const double* base, long elems) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(elems * 8), FP_BUF_FLAGS);
}
__device__ __forceinline__ double ldb(const double* base, long elems, unsigned byteoff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(buf(base, elems), byteoff, 0, 0));
}
// A wave-uniform pointer the compiler must treat as redefined at this point,
// so that what derives from it (the per-variable buffer resources) is
// rebuilt at the use from a few scalar operations instead of being hoisted
// into long-lived scalar registers, which would spill into vector lanes.
__device__ __forceinline__ const double* rebase(const double* p) {
    asm volatile("" : "+s"(p));
    return p;
}
__device__ __forceinline__ double* rebase(double* p) {
    asm volatile("" : "+s"(p));
    return p;
}

typedef unsigned int u32x2_t __attribute__((__vector_size__(2 * sizeof(unsigned int))));
__device__ __forceinline__ void stb(double* base, long elems, unsigned byteoff, double x) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, x), buf(base, elems), byteoff, 0, 0);
}

// The epilogue split in two, so that its loads can be issued early (before
// the face computation) and its stores done late: epi_load reads what the
// mode needs at node `off`, epi_store applies the same arithmetic as
// epilogue().
template <int NV>
struct EpiPre {
    double R[NV], qin[NV], qn[NV], V;
};

// (own_qv: the caller supplies 1/J and the stage input itself, from values
// it has staged already)
// (buffer loads and stores: one 32-bit byte offset per lane serves every
// variable array, whose base goes into the wave-uniform resource)
template <int NV>
__device__ __forceinline__ void epi_load(const EpiK& ep, long vol, long off, EpiPre<NV>& p,
                                         bool own_qv = false) {
    if (ep.mode == EPI_FIRST) return;
    const unsigned bo = (unsigned)off * 8u;
    const double* R = rebase(ep.R);
#pragma unroll
    for (int v = 0; v < NV; ++v) p.R[v] = ldb(R + v * vol, vol, bo);
    if (ep.mode == EPI_MID) return;
    if (!own_qv) p.V = ldb(rebase(ep.metV), vol, bo);
    if (ep.mode == EPI_LAST_RES) return;
    if (!own_qv) {
        const double* qin = rebase(ep.qin);
#pragma unroll
        for (int v = 0; v < NV; ++v) p.qin[v] = ldb(qin + v * vol, vol, bo);
    }
    if (ep.stage0) return;
    const double* qn = rebase(ep.qn);
#pragma unroll
    for (int v = 0; v < NV; ++v) p.qn[v] = ldb(qn + v * vol, vol, bo);
}

// The same epilogue with its mode fixed to MID (for a sweep that is never
// the last of a stage), so that no final-epilogue code is compiled in.
__device__ __forceinline__ EpiK epi_mid(const EpiK& ep) {
    EpiK e = ep;
    e.mode = EPI_MID;
    return e;
}

template <int NV>
__device__ __forceinline__ void epi_store(const EpiK& ep, long vol, long off, const EpiPre<NV>& p,
                                          const double (&d)[NV]) {
    const unsigned bo = (unsigned)off * 8u;
    if (ep.mode == EPI_FIRST) {
        double* R = rebase(ep.R);
#pragma unroll
        for (int v = 0; v < NV; ++v) stb(R + v * vol, vol, bo, -d[v]);
    } else if (ep.mode == EPI_MID) {
        double* R = rebase(ep.R);
#pragma unroll
        for (int v = 0; v < NV; ++v) stb(R + v * vol, vol, bo, p.R[v] - d[v]);
    } else if (ep.mode == EPI_LAST_RES) {
        const double J = 1.0 / p.V;  // one division per node, not one per variable
        double* out = rebase(ep.out);
#pragma unroll
        for (int v = 0; v < NV; ++v) stb(out + v * vol, vol, bo, (p.R[v] - d[v]) * J);
    } else {
        const double J = 1.0 / p.V;
        double* out = rebase(ep.out);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double k = (p.R[v] - d[v]) * J;
            const double u = p.qin[v] + ep.dt * k;
            stb(out + v * vol, vol, bo, ep.stage0 ? u : ep.a * p.qn[v] + ep.b * u);
        }
    }
}

// Reads the stencil of face i+1/2 of one grid line along axis DIR: slot r
// holds node i-3+r.  Periodic axes wrap to the image inside the interior;
// frozen axes read the ghost layers of the same array (the RK3 driver copies
// the caller's frozen ghost values into its stage arrays).  Metrics are read
// directly: fp_metrics fills their ghost layers.
template <int DIM, int DIR>
struct LineLoader {
    const double* __restrict__ met;
    const double* q;
    long vol;       // elements per variable
    unsigned lb;    // element offset of node 0 of the line
    int sd;         // element stride along the line
    int i;          // the face is i+1/2
    int nd;         // interior nodes along the line
    int per;        // periodic axis

    __device__ __forceinline__ LineLoader(const GeoK& G, const double* met_, const double* q_,
                                          long lb_, int i_)
        : met(met_), q(q_), vol(G.vol), lb((unsigned)lb_), sd((int)G.sd[DIR]), i(i_),
          nd(G.n[DIR]), per(G.bc[DIR] == 0) {}

    // A copy whose loads cannot be hoisted above, or merged with loads
    // before, the computation of `dep`: the line offset passes through an
    // empty asm that takes `dep` as input.  This bounds the live range of the
    // stencil values to one phase of the face computation.
    __device__ __forceinline__ LineLoader after(double dep) const {
        LineLoader c = *this;
        asm volatile("" : "+v"(c.lb) : "v"(dep));
        return c;
    }

    __device__ __forceinline__ void slot(int r, double (&qv)[DIM + 2], double& V,
                                         double (&s)[DIM]) const {
        constexpr int NMET = DIM == 3 ? 10 : 5;
        const int t = i - 3 + r;
        int tt = t;
        if (per) tt = t < 0 ? t + nd : (t >= nd ? t - nd : t);
        const unsigned off = (lb + (unsigned)(tt * sd)) * 8u;
        const unsigned moff = (lb + (unsigned)(t * sd)) * 8u;
#pragma unroll
        for (int v = 0; v < DIM + 2; ++v) qv[v] = ldb(q + v * vol, vol, off);
        V = ldb(met + (NMET - 1) * vol, vol, moff);
#pragma unroll
        for (int c = 0; c < DIM; ++c) s[c] = ldb(met + (DIR * DIM + c) * vol, vol, moff);
    }
};

template <int PREC>
using char_t = typename std::conditional<PREC == 1, float, double>::type;

// One dword per lane from a variable array of `elems` doubles into LDS
// (buffer-to-LDS DMA: no registers hold the data; completion is tracked by
// the wave's vmcnt).  Lane l writes the dword at lds + 4 l.  The array's
// base goes into the wave-uniform resource, so the lane supplies only its
// 32-bit byte offset (no per-load 64-bit address arithmetic).
__device__ __forceinline__ void dma_dword(const double* var, long elems, void* lds, unsigned byteoff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(buf(var, elems), (__attribute__((address_space(3))) void*)lds, 4,
                                             byteoff, 0, 0, 0);
}

// The wave's index in its workgroup, as a value the compiler knows to be
// uniform across the wave (so what derives from it stays in scalar registers).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ---------------------------------------------------------------------------
// xi sweep
// ---------------------------------------------------------------------------
// The faces of all xi-lines of a block are numbered flat, F = L (n0+1) + f
// (line L, face f-1/2 of it).  A wave item takes W consecutive faces,
// F = (W-1) j + l for lane l < W, so consecutive items overlap by one face:
// lane l > 0 takes its left neighbour's flux by a lane shift and forms the
// flux difference of its node.  The stencil nodes of the item are staged in
// the wave's own LDS buffer by global-to-LDS DMA, indexed by the extended
// flat index e = L (n0+8) + x + 4 (line L with four extra nodes on each side,
// x = -4 .. n0+3): slot r (node f-4+r) of face F is entry e(F) + r with
// e(F) = L (n0+8) + f.  A window of W faces spans W + 7 (lines touched)
// entries; W is the largest width (at most 64) that fits NE entries.  The
// sweeps that run three waves per SIMD stage NE = 88 entries (W = 64 still
// for lines of 30 nodes and more): the workgroup's double buffers then take
// 50 KB and three workgroups fit a CU's LDS; the others stage 128.
template <int DIM, int NE_>
struct XLds {
    static constexpr int NE = NE_;          // staged entries per buffer
    static constexpr int NS = 2 * DIM + 3;  // q, 1/J, s_xi
    double b[2][NS][NE];                    // double buffer: current item, next item
};
__device__ __host__ constexpr int x_entries(int prec, int recon, int Y) {
    return FP_XWAVES(prec, recon, Y) == 3 ? 88 : 128;
}

__device__ __host__ __forceinline__ int x_window(int n0, int ne) {
    int W = 64;
    while (W > 2 && W + 7 * ((W + n0) / (n0 + 1) + 1) > ne) --W;
    return W;
}

// wave items of the xi sweep of one block (ne: the sweep's staged entries)
__device__ __host__ __forceinline__ long sweep_x_items(const int n[3], int ne) {
    const long total = (long)(n[0] + 1) * n[1] * n[2];
    const int W = x_window(n[0], ne);
    return (total - 1 + W - 2) / (W - 1);
}

// floor(k / d) for 0 <= k, d < 2^20, in single precision: exact, since
// (k + 1/2) / d is at least 1/(2 d) away from an integer and the rounding
// error of the product is below k / d * 2^-23.
__device__ __forceinline__ unsigned small_div(unsigned k, float inv_d) {
    return (unsigned)(((float)k + 0.5f) * inv_d);
}

// Line L0 + dL of the xi-lines, from the decomposition (a1, a2) of L0 over
// (n1, n2): (l1, l2) with l1 < n1.
__device__ __forceinline__ void line_step(unsigned a1, unsigned a2, unsigned dL, unsigned n1, unsigned& l1,
                                          unsigned& l2) {
    l1 = a1 + dL;
    l2 = a2;
    while (l1 >= n1) {
        l1 -= n1;
        ++l2;
    }
}

// The uniform geometry of xi item j.
struct XItem {
    unsigned F0, L0, f0, a1, a2, count;
};

__device__ __forceinline__ XItem x_item(const GeoK& G, long j, int W) {
    XItem it;
    const unsigned nf = (unsigned)G.n[0] + 1, ne = (unsigned)G.n[0] + 8, n1 = (unsigned)G.n[1];
    const unsigned total = nf * n1 * (unsigned)G.n[2];
    it.F0 = (unsigned)((W - 1) * j);
    it.L0 = it.F0 / nf;
    it.f0 = it.F0 - it.L0 * nf;
    it.a1 = it.L0 % n1;
    it.a2 = it.L0 / n1;
    const unsigned Fl = min(it.F0 + (unsigned)W - 1, total - 1);
    const unsigned Ll = Fl / nf;
    it.count = (Ll - it.L0) * ne + (Fl - Ll * nf) + 8 - it.f0;  // entries e(F0) .. e(Fl) + 7
    return it;
}

// Stage item j's stencil entries into buf (all 64 lanes; asynchronous).
template <int DIM, int NE>
__device__ __forceinline__ void x_stage(const GeoK& G, const double* __restrict__ met, const double* qs,
                                        long j, int W, double (*buf)[NE]) {
    constexpr int NV = DIM + 2;
    constexpr int NMET = DIM == 3 ? 10 : 5;
    const unsigned lane = threadIdx.x & 63;
    const unsigned n0 = (unsigned)G.n[0], ne = n0 + 8, n1 = (unsigned)G.n[1], n2 = (unsigned)G.n[2];
    const XItem it = x_item(G, j, W);
    const float inv_ne = 1.0f / (float)ne;
    const int g = G.g;
    const int per = G.bc[0] == 0;
    const unsigned np = (it.count + 31) / 32;
#pragma unroll
    for (int p = 0; p < (NE + 31) / 32; ++p) {
        if ((unsigned)p >= np) break;
        // a pass moves 32 entries (two lanes per entry); the last one may be
        // partial, and its lanes past the buffer's end must write nothing
        if (NE % 32 != 0 && 32u * p + (lane >> 1) >= (unsigned)NE) continue;
        const unsigned k = it.f0 + 32u * p + (lane >> 1);  // from the start of line L0's entries
        const unsigned dL = small_div(k, inv_ne);
        const int x = (int)(k - dL * ne) - 4;
        unsigned l1, l2;
        line_step(it.a1, it.a2, dL, n1, l1, l2);
        if (l2 >= n2) {  // entries past the last line are never read
            l1 = n1 - 1;
            l2 = n2 - 1;
        }
        const int xm = x < -g ? -g : (x > (int)n0 - 1 + g ? (int)n0 - 1 + g : x);
        int xq = xm;
        if (per) {
            xq = x < 0 ? x + (int)n0 : (x >= (int)n0 ? x - (int)n0 : x);
            xq = xq < 0 ? 0 : (xq > (int)n0 - 1 ? (int)n0 - 1 : xq);
        }
        const unsigned lb = (unsigned)G.base + l1 * (unsigned)G.sd[1] + l2 * (unsigned)G.sd[2];
        const unsigned oq = (lb + (unsigned)xq) * 8u + (lane & 1) * 4u;
        const unsigned om = (lb + (unsigned)xm) * 8u + (lane & 1) * 4u;
        const double* qp = rebase(qs);
        const double* mp = rebase(met);
#pragma unroll
        for (int v = 0; v < NV; ++v) dma_dword(qp + v * G.vol, G.vol, &buf[v][32 * p], oq);
        dma_dword(mp + (NMET - 1) * G.vol, G.vol, &buf[NV][32 * p], om);
#pragma unroll
        for (int c = 0; c < DIM; ++c) dma_dword(mp + c * G.vol, G.vol, &buf[NV + 1 + c][32 * p], om);
    }
}

// Stencil reads of one lane's xi face from the wave's staged entries.
template <int DIM, int NE>
struct XLoader {
    const double (*buf)[NE];
    unsigned ea;  // byte offset of entry e(F) in a variable row

    __device__ __forceinline__ XLoader after(double dep) const {
        XLoader c = *this;
        asm volatile("" : "+v"(c.ea) : "v"(dep));
        return c;
    }

    __device__ __forceinline__ void slot(int r, double (&qv)[DIM + 2], double& V,
                                         double (&s)[DIM]) const {
        const char* row = reinterpret_cast<const char*>(&buf[0][0]) + ea + r * 8;
#pragma unroll
        for (int v = 0; v < DIM + 2; ++v) qv[v] = *reinterpret_cast<const double*>(row + v * NE * 8);
        V = *reinterpret_cast<const double*>(row + (DIM + 2) * NE * 8);
#pragma unroll
        for (int c = 0; c < DIM; ++c) s[c] = *reinterpret_cast<const double*>(row + (DIM + 3 + c) * NE * 8);
    }
};

// Faces of item j from its staged entries, the lane-shift difference and
// the epilogue (all 64 lanes must call this: the lane shift).  The xi sweep
// comes first in a stage, so its epilogue is FIRST (ACC = false: R = -d,
// nothing to load) or MID (ACC = true: R -= d, after the viscous part or a
// caller's accumulation; R loads while the face is computed).
template <int DIM, int RECON, int Y, int PREC, bool ACC>
__device__ __forceinline__ void x_compute(const GeoK& G, const SchemeK& sk, const EpiK& ep, long j, int W,
                                          const double (*buf)[x_entries(PREC, RECON, Y)]) {
    constexpr int NV = DIM + 2;
    const unsigned lane = threadIdx.x & 63;
    const unsigned nf = (unsigned)G.n[0] + 1, ne = (unsigned)G.n[0] + 8;
    const unsigned total = nf * (unsigned)G.n[1] * (unsigned)G.n[2];
    const XItem it = x_item(G, j, W);
    const unsigned F = it.F0 + lane;
    const bool active = lane < (unsigned)W && F < total;
    double fl[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) fl[v] = 0.0;
    const unsigned k = it.f0 + lane;  // from the first face of line L0
    const unsigned dL = small_div(k, 1.0f / (float)nf);
    const unsigned f = k - dL * nf;
    // lane l > 0 writes node f - 1, between its face and lane l - 1's
    const bool writes = active && lane > 0 && f > 0;
    long noff = 0;
    EpiPre<NV> pre;
    if (writes) {
        unsigned l1, l2;
        line_step(it.a1, it.a2, dL, (unsigned)G.n[1], l1, l2);
        noff = G.base + (long)l1 * G.sd[1] + (long)l2 * G.sd[2] + (f - 1);
        if (ACC) epi_load<NV>(epi_mid(ep), G.vol, noff, pre);
    }
    if (active) {
        XLoader<DIM, x_entries(PREC, RECON, Y)> ld;
        ld.buf = buf;
        ld.ea = (dL * ne + f - it.f0) * 8u;
        face_flux<DIM, RECON, Y, char_t<PREC>>(ld, sk, fl);
    }
    double d[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v] = fl[v] - __shfl_up(fl[v], 1, 64);
    if (writes) {
        if (ACC) {
            epi_store<NV>(epi_mid(ep), G.vol, noff, pre, d);
        } else {
            double* R = rebase(ep.R);
#pragma unroll
            for (int v = 0; v < NV; ++v) stb(R + v * G.vol, G.vol, (unsigned)noff * 8u, -d[v]);
        }
    }
}

// Persistent xi sweep of one block: wave w of the grid takes items w,
// w + (waves of the grid), ..., staging the next item while it computes
// (ACC: the epilogue is MID, not FIRST; those kernels run at two waves per
// SIMD, the accumulator's registers do not fit three).
#define FP_XWAVES_ACC(PREC, RECON, Y, ACC) ((ACC) ? 2 : FP_XWAVES(PREC, RECON, Y))
template <int DIM, int RECON, int Y, int PREC, bool ACC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FP_XWAVES_ACC(PREC, RECON, Y, ACC),
                                                                     FP_XWAVES_ACC(PREC, RECON, Y, ACC))))
void k_sweep_x(GeoK G, SchemeK sk, const double* __restrict__ met, const double* qs, EpiK ep) {
    constexpr int NE = x_entries(PREC, RECON, Y);
    __shared__ XLds<DIM, NE> lds[4];
    XLds<DIM, NE>& L = lds[wave_id()];
    const long nw = (long)gridDim.x * 4;
    const long items = sweep_x_items(G.n, NE);
    const int W = x_window(G.n[0], NE);
    long j = (long)blockIdx.x * 4 + wave_id();
    int cur = 0;
    if (j < items) x_stage<DIM, NE>(G, met, qs, j, W, L.b[0]);
    for (; j < items; j += nw, cur ^= 1) {
        __builtin_amdgcn_s_waitcnt(0);  // item j's entries are in LDS
        asm volatile("" ::: "memory");
        if (j + nw < items) x_stage<DIM, NE>(G, met, qs, j + nw, W, L.b[cur ^ 1]);
        x_compute<DIM, RECON, Y, PREC, ACC>(G, sk, ep, j, W, L.b[cur]);
    }
}

// LDS of an eta / zeta sweep workgroup: a ring of stencil rows (the q, 1/J
// and s_DIR values of the workgroup's 64 lines at one node index along
// DIR), the four face fluxes of an iteration and the carried last flux of
// the previous one.
constexpr int wide_stencil(int recon, int Y) { return (recon == 2 || Y == 8) ? 1 : 0; }

// WIDE: the face reads slots 0..7 (nodes i-3 .. i+4: eighth-order metrics or
// WENO7), else slots 1..6 (nodes i-2 .. i+3).
template <int DIM, int WIDE>
struct WgLds {
    static constexpr int NV = DIM + 2;
    static constexpr int NS = 2 * DIM + 3;   // values per node: q, 1/J, s_DIR
    static constexpr int LO = WIDE ? 3 : 2;  // nodes below node i a face i+1/2 reads
    static constexpr int HI = WIDE ? 4 : 3;  // nodes above node i
    static constexpr int WIN = 4 + LO + HI;    // rows read by the four faces of an iteration
    static constexpr int RING = WIN + 4;       // plus the four rows prefetched for the next
    double ring[RING][NS][64];
    double flux[4][NV][64];  // the four faces of the current iteration
    double carry[NV][64];    // the last face of the previous iteration
};

// Stencil reads of face i+1/2 from the LDS ring: slot r (node i-3+r) is ring
// row (b0 + r) mod RING.
template <int DIM, int WIDE>
struct LdsLoader {
    using W = WgLds<DIM, WIDE>;
    const W* L;
    unsigned la;  // byte offset of this lane in a ring row
    int b0;       // ring row of slot 0, in [0, RING)

    __device__ __forceinline__ LdsLoader after(double dep) const {
        LdsLoader c = *this;
        asm volatile("" : "+v"(c.la) : "v"(dep));
        return c;
    }

    __device__ __forceinline__ void slot(int r, double (&qv)[DIM + 2], double& V,
                                         double (&s)[DIM]) const {
        int idx = b0 + r;
        idx = idx >= W::RING ? idx - W::RING : idx;
        const char* row = reinterpret_cast<const char*>(&L->ring[idx][0][0]) + la;
#pragma unroll
        for (int v = 0; v < DIM + 2; ++v) qv[v] = *reinterpret_cast<const double*>(row + v * 512);
        V = *reinterpret_cast<const double*>(row + (DIM + 2) * 512);
#pragma unroll
        for (int c = 0; c < DIM; ++c) s[c] = *reinterpret_cast<const double*>(row + (DIM + 3 + c) * 512);
    }
};

// eta / zeta sweeps: a workgroup of four waves owns 64 grid lines along DIR
// (consecutive in the flattened (i, other) index, so row loads are
// coalesced) and one segment [k0, k1) of S nodes of them; work item `item`
// of a block is (line block = item % lblocks, segment = item / lblocks).
// The stencil rows are staged in an LDS ring by global-to-LDS DMA, one row
// per wave per iteration, prefetched one iteration ahead.  Per iteration
// wave w evaluates the face f+1/2, f = k0 - 1 + 4 it + w, on its 64 lines
// from the ring, the fluxes go to LDS and wave w forms node f's difference
// F'_{f+1/2} - F'_{f-1/2}.  Every thread of the workgroup runs the same
// iterations and barriers.  A caller that reuses `L` for another item must
// synchronise the workgroup first.
template <int DIM, int DIR, int RECON, int Y, int PREC>
__device__ __forceinline__ void sweep_wg_item(const GeoK& G, const SchemeK& sk,
                                              const double* __restrict__ met, const double* qs,
                                              const EpiK& ep, int S, long item,
                                              WgLds<DIM, wide_stencil(RECON, Y)>& L) {
    using W = WgLds<DIM, wide_stencil(RECON, Y)>;
    constexpr int NV = DIM + 2;
    constexpr int NMET = DIM == 3 ? 10 : 5;
    constexpr int OTH = DIR == 1 ? 2 : 1;
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const long nlines = (long)G.n[0] * G.n[OTH];
    const long lblocks = (nlines + 63) / 64;
    const long lineblk = item % lblocks;
    const int seg = (int)(item / lblocks);
    const long line = lineblk * 64 + lane;
    const bool lane_ok = line < nlines;
    const int i = lane_ok ? (int)(line % G.n[0]) : 0;
    const int o = lane_ok ? (int)(line / G.n[0]) : 0;
    const long lb = G.base + i + (long)o * G.sd[OTH];
    // DMA: lane l moves dword (l & 1) of line 32 h + l / 2 (h = 0, 1) of the
    // block; lines past the end repeat the last one
    unsigned loff[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        long ln = lineblk * 64 + 32 * h + (lane >> 1);
        ln = ln < nlines ? ln : nlines - 1;
        const long off = G.base + ln % G.n[0] + (ln / G.n[0]) * G.sd[OTH];
        loff[h] = (unsigned)off * 8u + (unsigned)(lane & 1) * 4u;
    }
    const int nd = G.n[DIR];
    const int per = G.bc[DIR] == 0;
    const int sdD = (int)G.sd[DIR];
    const long vol = G.vol;
    const int k0 = seg * S;
    const int k1 = min(k0 + S, nd);
    const int iters = (k1 - k0 + 1 + 3) / 4;  // faces k0-1/2 .. k1-1/2
    const int tb = k0 - 1 - W::LO;            // node index of ring row 0
    const int tmax = k1 - 1 + W::HI;          // last row any needed face reads
    // a final epilogue takes node f's stage input and 1/J from its ring row
    // (the stage input is the array this sweep reads, ep.qin == qs, and 1/J
    // the metric array's last component, in every caller) instead of memory
    constexpr bool own_qv = true;
    auto load_row = [&](int t) {
        if (t > tmax) return;
        const int slot = (t - tb) % W::RING;
        int tt = t;
        if (per) tt = t < 0 ? t + nd : (t >= nd ? t - nd : t);
        const unsigned qo = (unsigned)(tt * sdD) * 8u, mo = (unsigned)(t * sdD) * 8u;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double* qp = rebase(qs);
            const double* mp = rebase(met);
#pragma unroll
            for (int v = 0; v < NV; ++v) dma_dword(qp + v * vol, vol, &L.ring[slot][v][32 * h], loff[h] + qo);
            dma_dword(mp + (NMET - 1) * vol, vol, &L.ring[slot][NV][32 * h], loff[h] + mo);
#pragma unroll
            for (int c = 0; c < DIM; ++c)
                dma_dword(mp + (DIR * DIM + c) * vol, vol, &L.ring[slot][NV + 1 + c][32 * h], loff[h] + mo);
        }
    };
    for (int r = w; r < W::WIN; r += 4) load_row(tb + r);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        const int f = k0 - 1 + 4 * it + w;
        if (it + 1 < iters) load_row(tb + W::WIN + 4 * it + w);  // a row of the next iteration
        // this wave's node f: its epilogue operands load while the face is
        // computed (in FP64 WENO the zeta sweep then spills a few registers,
        // still faster than waiting for the loads after the face); 1/J and
        // the stage input of node f are in its ring row already
        const bool mine = lane_ok && f >= k0 && f < k1;
        const long noff = lb + (long)f * G.sd[DIR];
        EpiPre<NV> pre;
        if (mine) epi_load<NV>(ep, G.vol, noff, pre, own_qv);
        double F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = 0.0;
        if (lane_ok && f < k1) {
            LdsLoader<DIM, wide_stencil(RECON, Y)> ld;
            ld.L = &L;
            ld.la = (unsigned)lane * 8u;
            ld.b0 = (f - 3 - tb + W::RING) % W::RING;
            face_flux<DIM, RECON, Y, char_t<PREC>>(ld, sk, F);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) L.flux[w][v][lane] = F[v];
        __syncthreads();
        // FP32-mixed: the stores go after the second barrier, so that its
        // wait does not hold for their completion (they complete while the
        // next face is computed); FP64 stores before it, as holding the
        // epilogue operands across the barrier would spill its registers
        constexpr bool late_store = sizeof(char_t<PREC>) == 4;
        double d[NV];
        if (mine) {
            const double* prev = w > 0 ? &L.flux[w - 1][0][0] : &L.carry[0][0];
#pragma unroll
            for (int v = 0; v < NV; ++v) d[v] = F[v] - prev[v * 64 + lane];
            if (own_qv && ep.mode >= EPI_LAST_RES) {
                // node f's ring row (not overwritten before the next
                // iteration's barrier: the prefetched rows take other slots)
                const int slot = (f - tb) % W::RING;
                pre.V = L.ring[slot][NV][lane];
#pragma unroll
                for (int v = 0; v < NV; ++v) pre.qin[v] = L.ring[slot][v][lane];
            }
            if (!late_store) epi_store<NV>(ep, G.vol, noff, pre, d);
        }
        __builtin_amdgcn_s_waitcnt(0);  // this wave's row DMA has landed
        __syncthreads();                // every row of the next iteration is in LDS
        // the next iteration's first face needs this iteration's last flux;
        // the barrier above ended every read of the carry
        if (w == 3) {
#pragma unroll
            for (int v = 0; v < NV; ++v) L.carry[v][lane] = F[v];
        }
        if (late_store && mine) epi_store<NV>(ep, G.vol, noff, pre, d);
    }
}

// Work items (workgroups) of the eta / zeta sweep of one block.
inline long sweep_wg_items(const int n[3], int dir, int S) {
    const int oth = dir == 1 ? 2 : 1;
    const long lblocks = ((long)n[0] * n[oth] + 63) / 64;
    return lblocks * ((n[dir] + S - 1) / S);
}

// One launch of the eta / zeta sweep of one block, with its epilogue mode
// (EPI_*) fixed at compile time, as in the batched sweeps, so that only that
// epilogue's registers are allocated.
template <int DIM, int DIR, int RECON, int Y, int PREC, int MODE>
__global__ __launch_bounds__(256) FP_SWEEP_ATTR void k_sweep_wg(GeoK G, SchemeK sk,
                                                                const double* __restrict__ met,
                                                                const double* qs, EpiK ep, int S) {
    __shared__ WgLds<DIM, wide_stencil(RECON, Y)> lds;
    EpiK e = ep;
    e.mode = MODE;
    sweep_wg_item<DIM, DIR, RECON, Y, PREC>(G, sk, met, qs, e, S, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// global Lax-Friedrichs speeds
// ---------------------------------------------------------------------------

// The speeds live in sets of three directions; direction d of a set takes
// the three doubles at 16 d (one 128-byte line per direction, so the
// reductions of different directions do not contend for one line).
constexpr int kGlfDirStride = 16;
constexpr int kGlfSetStride = 3 * kGlfDirStride;
// faces per thread of the reduction (neighbours along the face direction)
constexpr int kGlfSeg = 2;

// Zero one speed set (a template: this header is compiled into several objects).
template <int DIM>
__global__ void k_glf_reset(unsigned long long* set) {
    if (threadIdx.x < 9) set[kGlfDirStride * (threadIdx.x / 3) + threadIdx.x % 3] = 0ull;
}

// velocity and sound speed of the node at `off`
template <int DIM>
__device__ __forceinline__ void glf_node(const double* __restrict__ q, long vol, long off, double gamma,
                                         double* u, double& cs) {
    const double rho = q[off];
    double k2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double mc = q[(1 + c) * vol + off];
        u[c] = mc / rho;
        k2 += mc * u[c];
    }
    const double p = (gamma - 1.0) * (q[(DIM + 1) * vol + off] - 0.5 * k2);
    cs = sqrt(gamma * p / rho);
}

// The largest local Lax-Friedrichs speed over every face of every direction
// (faces f + 1/2, f = -1 .. n_d - 1, of every interior line), per field class
// (u_n - c, u_n, u_n + c): at each face the metric vector and 1/J are
// interpolated (order Y) as for the face's reference state, n = s_f/|s_f|,
// sigma = |s_f|/(1/J)_f, and the speeds sigma |n . u_m + kappa c_m| are
// maximised over the stencil nodes m = f - LO .. f + LO + 1.  As in the
// sweeps, the state's index wraps into the interior on a periodic axis (its
// ghost layers are not filled) and the metrics are read in place.
//
// Blocks [d bpd, (d + 1) bpd) take direction d.  A thread takes kGlfSeg
// neighbouring faces of one line and evaluates the velocity and sound speed
// of each node of their stencils once; consecutive threads take consecutive
// face pairs along the line for xi and neighbouring lines (contiguous in
// memory) for eta and zeta.  Each block reduces its maxima and folds them
// into `set` with one integer atomic max per class (non-negative doubles
// order as their bit patterns do): few large blocks, since atomics on one
// cache line serialise.  Block 0 also zeroes `next` (the set the following
// reduction folds into; NULL: none).
template <int DIM, int Y, int LO>
__global__ __launch_bounds__(1024) void k_glf(GeoK G, double gamma, const double* __restrict__ met,
                                              const double* __restrict__ q, unsigned long long* set,
                                              unsigned long long* next, int bpd) {
    constexpr int NMET = DIM == 3 ? 10 : 5;
    constexpr int NW = kGlfSeg + 2 * LO + 1;  // stencil nodes of one segment
    const int d = blockIdx.x / bpd, bb = blockIdx.x % bpd;
    if (next && blockIdx.x == 0 && threadIdx.x < 9)
        next[kGlfDirStride * (threadIdx.x / 3) + threadIdx.x % 3] = 0ull;
    const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
    const long n1 = G.n[e1], n12 = n1 * G.n[e2];
    const int nd = G.n[d];
    const int nseg = (nd + kGlfSeg) / kGlfSeg;  // segments of the n_d + 1 faces of a line
    const long total = (long)nseg * n12;
    const long sdd = G.sd[d];
    const bool per = G.bc[d] == 0;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (long t = (long)bb * blockDim.x + threadIdx.x; t < total; t += (long)bpd * blockDim.x) {
        long r;
        int sg;
        if (d == 0) {
            sg = (int)(t % nseg);
            r = t / nseg;
        } else {
            r = t % n12;
            sg = (int)(t / n12);
        }
        const int f0 = sg * kGlfSeg - 1;
        const long line = G.base + (r % n1) * G.sd[e1] + (r / n1) * G.sd[e2];
        double u[NW][DIM], cs[NW];
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            // nodes past the last face's stencil are never read: clamp them
            int p = min(f0 - LO + j, nd + LO);
            if (per) p = p < 0 ? p + nd : (p >= nd ? p - nd : p);
            glf_node<DIM>(q, G.vol, line + (long)p * sdd, gamma, u[j], cs[j]);
        }
#pragma unroll
        for (int j = 0; j < kGlfSeg; ++j) {
            const int f = f0 + j;
            if (f >= nd) break;
            double Vf = 0.0, sf[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) sf[c] = 0.0;
#pragma unroll
            for (int m = 0; m < Y; ++m) {
                const long off = line + (long)(f - Y / 2 + 1 + m) * sdd;
                const double w = iw<Y>(m + 4 - Y / 2);
                Vf += w * met[(NMET - 1) * G.vol + off];
#pragma unroll
                for (int c = 0; c < DIM; ++c) sf[c] += w * met[(d * DIM + c) * G.vol + off];
            }
            double s2 = 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s2 += sf[c] * sf[c];
            const double sn = sqrt(s2);
            const double sigma = sn / Vf;
            double n[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) n[c] = sf[c] / sn;
#pragma unroll
            for (int m = 0; m <= 2 * LO + 1; ++m) {
                double un = 0.0;
#pragma unroll
                for (int c = 0; c < DIM; ++c) un += n[c] * u[j + m][c];
                m0 = fmax(m0, sigma * fabs(un - cs[j + m]));
                m1 = fmax(m1, sigma * fabs(un));
                m2 = fmax(m2, sigma * fabs(un + cs[j + m]));
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m0 = fmax(m0, __shfl_xor(m0, o));
        m1 = fmax(m1, __shfl_xor(m1, o));
        m2 = fmax(m2, __shfl_xor(m2, o));
    }
    __shared__ double red[3][16];
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = m0;
        red[1][w] = m1;
        red[2][w] = m2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        double v = 0.0;
        for (int i = 0; i < nw; ++i) v = fmax(v, red[k][i]);
        atomicMax(set + kGlfDirStride * d + k, (unsigned long long)__double_as_longlong(v));
    }
}

// ---------------------------------------------------------------------------
// batches: many blocks (of one dimensionality and scheme) in shared launches
// ---------------------------------------------------------------------------

// One block of a batch as the batched kernels see it.
struct BBlock {
    GeoK G;
    const double* met;
    double* q;  // Q^n, and the output of RK stage 3
    double* A;  // RK stage registers and residual accumulator (the workspace)
    double* B;
    double* R;
    double dt;
    int S[3];  // eta / zeta segment lengths
};

// Kinds of work items of a batched RK step.
enum { BK_X = 0, BK_ETA = 1, BK_ZETA = 2, BK_GHOST = 3, BK_KINDS = 4 };

// An interface between two blocks of a batch: the ghost layers of block a
// on `side` (0 low, 1 high) of `axis` are the interior layers of block b
// next to its opposite side (the blocks share the other axes' extents and
// orientation).
struct LinkK {
    int a, b, axis, side;
};

// Work-item table of a batch, in device memory.  The number of blocks and
// the prefix sums are read by the kernels at run time, so a captured graph
// stays valid when the table's contents change:
//   *nblk                      blocks in use;
//   start[k * (cap + 1) + b]   first item of block b in kind k; entry nblk is
//                              the kind's total;
//   blk[b]                     the block.
struct BTab {
    const int* nblk;
    const long* start;
    const BBlock* blk;
    int cap;
};

// The order of the blocks within a kind's work list: position n of kind k
// holds block kind_order(...)[n] (the list of a kind may put its blocks in
// any order; the eta / zeta lists put the blocks with the longest items
// first, so that the cyclic assignment of items to workgroups balances).
// The array follows the prefix sums in the same table.
__device__ __forceinline__ const int* kind_order(const long* t_start, int cap, int kind) {
    return reinterpret_cast<const int*>(t_start + BK_KINDS * (cap + 1)) + kind * cap;
}

// Block of `item` at or after block b, for items that only increase.
__device__ __forceinline__ int advance_block(const long* st, int nblk, int b, long item) {
    while (b + 1 < nblk && st[b + 1] <= item) ++b;
    return b;
}

// Largest b in [0, nblk) with st[b] <= item (blocks without items of a kind
// have st[b] == st[b + 1] and are skipped).
__device__ __forceinline__ int find_block(const long* st, int nblk, long item) {
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st[mid] <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ const double* stage_in(const BBlock& b, int stage) {
    return stage == 0 ? b.q : (stage == 1 ? b.A : b.B);
}

// The epilogue of a sweep of RK stage `stage` (TVD RK3 in Shu-Osher form:
// stage 1 writes A, stage 2 B, stage 3 q), the same values the single-block
// driver uses.
__device__ __forceinline__ EpiK stage_epi(const BBlock& b, int stage, int mode, int ndim) {
    EpiK e;
    e.mode = mode;
    e.stage0 = stage == 0;
    e.R = b.R;
    e.out = stage == 0 ? b.A : (stage == 1 ? b.B : b.q);
    e.metV = b.met + (ndim == 3 ? 9 : 4) * b.G.vol;
    e.qin = stage_in(b, stage);
    e.qn = b.q;
    e.dt = b.dt;
    e.a = stage == 0 ? 0.0 : (stage == 1 ? 3.0 / 4.0 : 1.0 / 3.0);
    e.b = stage == 0 ? 1.0 : (stage == 1 ? 1.0 / 4.0 : 2.0 / 3.0);
    return e;
}

// Persistent batched xi sweep of one RK stage: wave w of the grid takes the
// batch's wave items w, w + (waves of the grid), ..., staging the next item
// (possibly of another block) while it computes.
template <int DIM, int RECON, int Y, int PREC>
__global__ __launch_bounds__(256) FP_XSWEEP_ATTR(PREC, RECON, Y) void kb_sweep_x(const int* __restrict__ t_nblk,
                                                                const long* __restrict__ t_start,
                                                                const BBlock* __restrict__ t_blk, int cap,
                                                                SchemeK sk, int stage) {
    constexpr int NE = x_entries(PREC, RECON, Y);
    __shared__ XLds<DIM, NE> lds[4];
    XLds<DIM, NE>& L = lds[wave_id()];
    const int nblk = *t_nblk;
    const long* __restrict__ st = t_start + BK_X * (cap + 1);
    const long total = st[nblk];
    const int* __restrict__ ord = kind_order(t_start, cap, BK_X);
    const long nw = (long)gridDim.x * 4;
    long item = (long)blockIdx.x * 4 + wave_id();
    int cur = 0;
    int b = 0;
    if (item < total) {
        b = find_block(st, nblk, item);
        const BBlock& B = t_blk[ord[b]];
        x_stage<DIM, NE>(B.G, B.met, stage_in(B, stage), item - st[b], x_window(B.G.n[0], NE), L.b[0]);
    }
    for (; item < total; item += nw, cur ^= 1) {
        __builtin_amdgcn_s_waitcnt(0);
        asm volatile("" ::: "memory");
        int bn = b;
        if (item + nw < total) {
            bn = advance_block(st, nblk, b, item + nw);
            const BBlock& N = t_blk[ord[bn]];
            x_stage<DIM, NE>(N.G, N.met, stage_in(N, stage), item + nw - st[bn], x_window(N.G.n[0], NE),
                             L.b[cur ^ 1]);
        }
        const BBlock& B = t_blk[ord[b]];
        const EpiK ep = stage_epi(B, stage, EPI_FIRST, DIM);
        x_compute<DIM, RECON, Y, PREC, false>(B.G, sk, ep, item - st[b], x_window(B.G.n[0], NE), L.b[cur]);
        b = bn;
    }
}

// Persistent batched eta / zeta sweep of one RK stage; the last direction
// applies the RK3 update.
template <int DIM, int DIR, int RECON, int Y, int PREC>
__global__ __launch_bounds__(256) FP_SWEEP_ATTR void kb_sweep_wg(const int* __restrict__ t_nblk,
                                                                 const long* __restrict__ t_start,
                                                                 const BBlock* __restrict__ t_blk, int cap,
                                                                 SchemeK sk, int stage) {
    __shared__ WgLds<DIM, wide_stencil(RECON, Y)> lds;
    constexpr int KIND = DIR == 1 ? BK_ETA : BK_ZETA;
    constexpr int MODE = DIR == DIM - 1 ? EPI_LAST_RK : EPI_MID;
    const int nblk = *t_nblk;
    const long* __restrict__ st = t_start + KIND * (cap + 1);
    const long total = st[nblk];
    const int* __restrict__ ord = kind_order(t_start, cap, KIND);
    int b = blockIdx.x < total ? find_block(st, nblk, blockIdx.x) : 0;
    for (long item = blockIdx.x; item < total; item += gridDim.x) {
        b = advance_block(st, nblk, b, item);
        const BBlock& B = t_blk[ord[b]];
        const EpiK ep = stage_epi(B, stage, MODE, DIM);
        sweep_wg_item<DIM, DIR, RECON, Y, PREC>(B.G, sk, B.met, stage_in(B, stage), ep, B.S[DIR],
                                                item - st[b], lds);
        __syncthreads();  // the next item rewrites the LDS ring
    }
}

// Every face of direction DIR, one lane per face, lanes along i (coalesced):
// the face fluxes of fp_face_fluxes.
template <int DIM, int DIR, int RECON, int Y, int PREC>
__global__ __launch_bounds__(256) FP_SWEEP_ATTR void k_face_flux(GeoK G, SchemeK sk,
                                                                 const double* __restrict__ met,
                                                                 const double* qs, double* out) {
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
    const LineLoader<DIM, DIR> ld(G, met, qs, lb, c[DIR] - 1);
    double fl[NV];
    face_flux<DIM, RECON, Y, char_t<PREC>>(ld, sk, fl);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * total + tid] = fl[v];
}

// ---------------------------------------------------------------------------
// launch helpers (defined in the instantiation units)
// ---------------------------------------------------------------------------

// Launch timing of an instrumented step: after each launch the host records
// an event on the stream and the launch's kind (kinds as fp_profile_step
// reports them).  The first error stops the recording.
enum {
    PK_XI = 0, PK_ETA = 1, PK_ZETA = 2, PK_GHOST = 3, PK_GLF = 5, PK_BC = 6, PK_VFLUX = 7, PK_VDIV = 8,
    PK_GLF_RESET = 9
};
struct Probe {
    hipEvent_t* ev;  // ev[0] is recorded before the first launch; ev[i + 1] after launch i
    int32_t* kind;
    int n, cap;
    hipError_t err;
};
inline void probe_mark(Probe* p, int kind, hipStream_t s) {
    if (!p || p->err != hipSuccess) return;
    if (p->n >= p->cap) {
        p->err = hipErrorInvalidValue;
        return;
    }
    p->err = hipGetLastError();
    if (p->err == hipSuccess) p->err = hipEventRecord(p->ev[p->n + 1], s);
    if (p->err == hipSuccess) p->kind[p->n++] = kind;
}

struct SweepArgs {
    GeoK G;
    SchemeK sk;
    const double* met;
    const double* qs;
    EpiK ep_first, ep_mid, ep_last;
    int S[3];
    int nseg[3];
    int glf;  // 1: reduce the global LF speeds of the stage input into sk.glf first
    double* glf_next;  // the speed set the reduction zeroes for the next stage (or NULL)
    Probe* probe;      // instrumented step (or NULL)
};

// one full residual evaluation (all sweeps) of the given instantiation
using stage_fn = hipError_t (*)(const SweepArgs&, hipStream_t);
using faceflux_fn = hipError_t (*)(const GeoK&, const SchemeK&, const double*, const double*,
                                   double*, hipStream_t);
// one direction sweep of the given instantiation with epilogue `ep`
using dir_fn = hipError_t (*)(const SweepArgs&, int dir, const EpiK& ep, hipStream_t);

// one RK stage of a batch part: the xi, eta (and zeta) persistent sweeps,
// grid[k] workgroups for sweep kind k; only >= 0 launches that kind alone
using batch_stage_fn = hipError_t (*)(const BTab&, const SchemeK&, int stage, const int grid[3],
                                      int only, hipStream_t);
// resident workgroups per CU of the batched sweep of kind k
using batch_occ_fn = int (*)(int kind);

stage_fn get_stage_fn(int ndim, int recon, int Y, int prec);
batch_stage_fn get_batch_stage_fn(int ndim, int recon, int Y, int prec);
batch_occ_fn get_batch_occ_fn(int ndim, int recon, int Y, int prec);
faceflux_fn get_faceflux_fn(int ndim, int dir, int recon, int Y, int prec);
dir_fn get_dir_fn(int ndim, int recon, int Y, int prec);

}  // namespace fpk
