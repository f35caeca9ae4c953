// fp_util_kernels.hpp -- setup and utility kernels (metrics, periodic ghost
// copy, CFL limit, state check).  Included by fp_api.hip only.
#pragma once
#include "fp_kernels.hpp"

namespace fpk {

// ---------------------------------------------------------------------------
// symmetric conservative metrics (setup)
// ---------------------------------------------------------------------------

struct CGeoK {
    int gc;
    long csd[3];
    long cvol;
    long cbase;  // offset of node (0,0,0) in the coordinate arrays
};

// antisymmetric central first-derivative weights c_m, m = 1..Y/2:
// D f = sum_m c_m (f_{+m} - f_{-m})
template <int Y>
__device__ __forceinline__ double dcoef(int m) {
    if constexpr (Y == 2) {
        return 0.5;
    } else if constexpr (Y == 4) {
        return m == 1 ? 8.0 / 12.0 : -1.0 / 12.0;
    } else if constexpr (Y == 6) {
        return m == 1 ? 45.0 / 60.0 : (m == 2 ? -9.0 / 60.0 : 1.0 / 60.0);
    } else {
        return m == 1 ? 672.0 / 840.0 : (m == 2 ? -168.0 / 840.0 : (m == 3 ? 32.0 / 840.0 : -3.0 / 840.0));
    }
}

template <int Y>
struct Coord {
    const double* xyz;
    CGeoK C;
    __device__ __forceinline__ double X(int c, long off) const { return xyz[c * C.cvol + off]; }
    // derivative of coordinate c along axis e at the node with offset off
    __device__ __forceinline__ double D(int c, int e, long off) const {
        double s = 0.0;
#pragma unroll
        for (int m = 1; m <= Y / 2; ++m)
            s += dcoef<Y>(m) * (X(c, off + m * C.csd[e]) - X(c, off - m * C.csd[e]));
        return s;
    }
    // P_e = a_e b - a b_e (the pairing of eq. JBabc)
    __device__ __forceinline__ double P(int a, int b, int e, long off) const {
        return D(a, e, off) * X(b, off) - X(a, off) * D(b, e, off);
    }
    // s_{d,c}: with (e, f) = (d+1, d+2) and (a, b) = (c+1, c+2) cyclically,
    // s_{d,c} = 1/2 [ (a_e b - a b_e)_f - (a_f b - a b_f)_e ]
    __device__ __forceinline__ double s3(int d, int c, long off) const {
        const int e = (d + 1) % 3, f = (d + 2) % 3;
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        double sf = 0.0, se = 0.0;
#pragma unroll
        for (int m = 1; m <= Y / 2; ++m) {
            sf += dcoef<Y>(m) * (P(a, b, e, off + m * C.csd[f]) - P(a, b, e, off - m * C.csd[f]));
            se += dcoef<Y>(m) * (P(a, b, f, off + m * C.csd[e]) - P(a, b, f, off - m * C.csd[e]));
        }
        return 0.5 * (sf - se);
    }
    // x . s_d at a node (the flux of eq. JB)
    __device__ __forceinline__ double xs3(int d, long off) const {
        return X(0, off) * s3(d, 0, off) + X(1, off) * s3(d, 1, off) + X(2, off) * s3(d, 2, off);
    }
};

template <int DIM, int Y>
__global__ __launch_bounds__(128) void k_metrics(GeoK G, CGeoK C, const double* __restrict__ xyz,
                                                  double* met, int lo0, int lo1, int lo2, int c0,
                                                  int c1, int c2) {
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long)c0 * c1 * c2) return;
    const int i = lo0 + (int)(tid % c0);
    const int j = lo1 + (int)((tid / c0) % c1);
    const int k = lo2 + (int)(tid / ((long)c0 * c1));
    const Coord<Y> X{xyz, C};
    const long co = C.cbase + i + j * C.csd[1] + (long)k * C.csd[2];
    const long mo = G.base + i + j * G.sd[1] + (long)k * G.sd[2];
    if constexpr (DIM == 3) {
#pragma unroll 1
        for (int d = 0; d < 3; ++d)
#pragma unroll 1
            for (int c = 0; c < 3; ++c) met[(3 * d + c) * G.vol + mo] = X.s3(d, c, co);
        double J = 0.0;
#pragma unroll 1
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
#pragma unroll 1
            for (int m = 1; m <= Y / 2; ++m)
                s += dcoef<Y>(m) * (X.xs3(d, co + m * C.csd[d]) - X.xs3(d, co - m * C.csd[d]));
            J += s;
        }
        met[9 * G.vol + mo] = J / 3.0;
    } else {
        met[0 * G.vol + mo] = X.D(1, 1, co);
        met[1 * G.vol + mo] = -X.D(0, 1, co);
        met[2 * G.vol + mo] = -X.D(1, 0, co);
        met[3 * G.vol + mo] = X.D(0, 0, co);
        // 1/J = 1/2 [ (x y_eta - y x_eta)_xi + (y x_xi - x y_xi)_eta ]
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int m = 1; m <= Y / 2; ++m) {
            const long p = co + m * C.csd[0], q = co - m * C.csd[0];
            a += dcoef<Y>(m) * ((X.X(0, p) * X.D(1, 1, p) - X.X(1, p) * X.D(0, 1, p)) -
                                (X.X(0, q) * X.D(1, 1, q) - X.X(1, q) * X.D(0, 1, q)));
            const long r = co + m * C.csd[1], s = co - m * C.csd[1];
            b += dcoef<Y>(m) * ((X.X(1, r) * X.D(0, 0, r) - X.X(0, r) * X.D(1, 0, r)) -
                                (X.X(1, s) * X.D(0, 0, s) - X.X(0, s) * X.D(1, 0, s)));
        }
        met[4 * G.vol + mo] = 0.5 * (a + b);
    }
}

// Periodic ghost layers of any [nvar][...] array: copy from the image.
__global__ __launch_bounds__(256) void k_periodic_fill(GeoK G, int ndim, int nvar, double* a) {
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= G.vol) return;
    int N[3];
    N[0] = G.n[0] + 2 * G.g;
    N[1] = G.n[1] + 2 * G.g;
    N[2] = ndim == 3 ? G.n[2] + 2 * G.g : 1;
    int p[3];
    p[0] = (int)(tid % N[0]) - G.g;
    p[1] = (int)((tid / N[0]) % N[1]) - G.g;
    p[2] = ndim == 3 ? (int)(tid / ((long)N[0] * N[1])) - G.g : 0;
    bool moved = false;
    for (int d = 0; d < ndim; ++d) {
        if (G.bc[d] == 0 && (p[d] < 0 || p[d] >= G.n[d])) {
            p[d] = ((p[d] % G.n[d]) + G.n[d]) % G.n[d];
            moved = true;
        }
    }
    if (!moved) return;
    const long src = G.base + p[0] + p[1] * G.sd[1] + (long)p[2] * G.sd[2];
    for (int v = 0; v < nvar; ++v) a[v * G.vol + tid] = a[v * G.vol + src];
}

// Nodes of the ghost slabs of the frozen axes: for each frozen axis d, the
// g layers on each side along d with the other coordinates interior (the
// only ghost nodes the sweeps read).
__host__ __device__ inline long frozen_slab_nodes(const GeoK& G, int ndim) {
    long tot = 0;
    for (int d = 0; d < ndim; ++d) {
        if (G.bc[d] == 0) continue;
        long c = 2L * G.g;
        for (int e = 0; e < ndim; ++e)
            if (e != d) c *= G.n[e];
        tot += c;
    }
    return tot;
}

// Copies slab node t (0 <= t < frozen_slab_nodes) of src into dst1 and dst2:
// the RK3 drivers give their stage registers the caller's boundary values.
__device__ __forceinline__ void frozen_ghost_node(const GeoK& G, int ndim, int nvar, const double* src,
                                                  double* dst1, double* dst2, long t) {
    for (int d = 0; d < ndim; ++d) {
        if (G.bc[d] == 0) continue;
        long c = 2L * G.g;
        for (int e = 0; e < ndim; ++e)
            if (e != d) c *= G.n[e];
        if (t >= c) {
            t -= c;
            continue;
        }
        const int ad = (int)(t % (2 * G.g));
        long rest = t / (2 * G.g);
        long off = G.base + (long)(ad < G.g ? ad - G.g : G.n[d] + ad - G.g) * G.sd[d];
        for (int e = 0; e < ndim; ++e) {
            if (e == d) continue;
            off += (rest % G.n[e]) * G.sd[e];
            rest /= G.n[e];
        }
        for (int v = 0; v < nvar; ++v) {
            const double x = src[v * G.vol + off];
            dst1[v * G.vol + off] = x;
            dst2[v * G.vol + off] = x;
        }
        return;
    }
}

__global__ __launch_bounds__(256) void k_frozen_ghosts(GeoK G, int ndim, int nvar,
                                                       const double* __restrict__ src,
                                                       double* __restrict__ dst1,
                                                       double* __restrict__ dst2) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < frozen_slab_nodes(G, ndim)) frozen_ghost_node(G, ndim, nvar, src, dst1, dst2, t);
}

// Batched form: one item = 256 slab nodes of one block.
__global__ __launch_bounds__(256) void kb_frozen_ghosts(const int* __restrict__ t_nblk,
                                                        const long* __restrict__ t_start,
                                                        const BBlock* __restrict__ t_blk, int cap, int ndim) {
    const int nblk = *t_nblk;
    const long* __restrict__ st = t_start + BK_GHOST * (cap + 1);
    const long total = st[nblk];
    int b = blockIdx.x < total ? find_block(st, nblk, blockIdx.x) : 0;
    for (long item = blockIdx.x; item < total; item += gridDim.x) {
        b = advance_block(st, nblk, b, item);
        const BBlock& B = t_blk[b];
        const long node = (item - st[b]) * 256 + threadIdx.x;
        if (node < frozen_slab_nodes(B.G, ndim))
            frozen_ghost_node(B.G, ndim, ndim + 2, B.q, B.A, B.B, node);
    }
}

// Interface exchange: for every link, the g ghost layers of block a on its
// side are copied from the interior layers of block b next to the opposite
// side.  which = 0, 1, 2: the state registers of RK stage 1 (q), 2 (A),
// 3 (B); which = 3: the metric arrays.  Node t of all links' ghost slabs
// (prefix sums lstart) per thread; lanes follow their link forward.
__global__ __launch_bounds__(256) void kb_halo(const int* __restrict__ t_nlink,
                                               const long* __restrict__ t_lstart,
                                               const LinkK* __restrict__ t_links,
                                               const BBlock* __restrict__ t_blk, int ndim, int which) {
    const int nl = *t_nlink;
    const long total = t_lstart[nl];
    int li = 0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        while (li + 1 < nl && t_lstart[li + 1] <= t) ++li;
        const LinkK L = t_links[li];
        const BBlock& A = t_blk[L.a];
        const BBlock& B = t_blk[L.b];
        const int g = A.G.g;
        long u = t - t_lstart[li];
        const int l = (int)(u % g);
        u /= g;
        long oa = A.G.base, ob = B.G.base;
        for (int e = 0; e < ndim; ++e) {
            if (e == L.axis) continue;
            const long c = u % A.G.n[e];
            u /= A.G.n[e];
            oa += c * A.G.sd[e];
            ob += c * B.G.sd[e];
        }
        const int ia = L.side ? A.G.n[L.axis] + l : -1 - l;
        const int ib = L.side ? l : B.G.n[L.axis] - 1 - l;
        oa += (long)ia * A.G.sd[L.axis];
        ob += (long)ib * B.G.sd[L.axis];
        if (which == 3) {
            double* dst = const_cast<double*>(A.met);
            const int nmet = ndim == 3 ? 10 : 5;
            for (int v = 0; v < nmet; ++v) dst[v * A.G.vol + oa] = B.met[v * B.G.vol + ob];
        } else {
            double* dst = which == 0 ? A.q : (which == 1 ? A.A : A.B);
            const double* src = which == 0 ? B.q : (which == 1 ? B.A : B.B);
            for (int v = 0; v < ndim + 2; ++v) dst[v * A.G.vol + oa] = src[v * B.G.vol + ob];
        }
    }
}

// ---------------------------------------------------------------------------
// CFL limit and state check
// ---------------------------------------------------------------------------

__global__ void k_dt_init(unsigned long long* bits) { *bits = 0ull; }

template <int DIM>
__global__ __launch_bounds__(256) void k_dt_reduce(GeoK G, double gamma,
                                                    const double* __restrict__ met,
                                                    const double* __restrict__ q,
                                                    unsigned long long* bits) {
    constexpr int NV = DIM + 2, NMET = DIM == 3 ? 10 : 5;
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long tot = (long)G.n[0] * G.n[1] * G.n[2];
    double val = 0.0;
    if (tid < tot) {
        const int i = (int)(tid % G.n[0]);
        const int j = (int)((tid / G.n[0]) % G.n[1]);
        const int k = (int)(tid / ((long)G.n[0] * G.n[1]));
        const long off = G.base + i + j * G.sd[1] + (long)k * G.sd[2];
        const double rho = q[off];
        double u[DIM], m2 = 0.0;
        for (int c = 0; c < DIM; ++c) {
            u[c] = q[(1 + c) * G.vol + off] / rho;
            m2 += q[(1 + c) * G.vol + off] * u[c];
        }
        const double p = (gamma - 1.0) * (q[(NV - 1) * G.vol + off] - 0.5 * m2);
        const double cs = sqrt(gamma * p / rho);
        double sum = 0.0;
        for (int d = 0; d < DIM; ++d) {
            double su = 0.0, ss = 0.0;
            for (int c = 0; c < DIM; ++c) {
                const double s = met[(d * DIM + c) * G.vol + off];
                su += s * u[c];
                ss += s * s;
            }
            sum += fabs(su) + cs * sqrt(ss);
        }
        val = sum / met[(NMET - 1) * G.vol + off];
    }
    __shared__ double red[256];
    red[threadIdx.x] = val;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(bits, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void k_dt_final(unsigned long long* bits, double cfl) {
    const double mx = __longlong_as_double((long long)*bits);
    *reinterpret_cast<double*>(bits) = cfl / mx;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_check_state(GeoK G, double gamma, const double* __restrict__ q,
                                                      int* flag) {
    constexpr int NV = DIM + 2;
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long tot = (long)G.n[0] * G.n[1] * G.n[2];
    if (tid >= tot) return;
    const int i = (int)(tid % G.n[0]);
    const int j = (int)((tid / G.n[0]) % G.n[1]);
    const int k = (int)(tid / ((long)G.n[0] * G.n[1]));
    const long off = G.base + i + j * G.sd[1] + (long)k * G.sd[2];
    double Q[NV];
    bool bad = false;
    for (int v = 0; v < NV; ++v) {
        Q[v] = q[v * G.vol + off];
        bad |= !isfinite(Q[v]);
    }
    double m2 = 0.0;
    for (int c = 0; c < DIM; ++c) m2 += Q[1 + c] * Q[1 + c];
    const double p = (gamma - 1.0) * (Q[NV - 1] - 0.5 * m2 / Q[0]);
    bad |= !(Q[0] > 0.0) || !(p > 0.0);
    if (bad) *flag = 1;
}

}  // namespace fpk
