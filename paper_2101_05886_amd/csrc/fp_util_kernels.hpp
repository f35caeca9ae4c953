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
        // the layer ad (both sides) and the transverse indices c1 (axis e1),
        // c2 (axis e2, 3D): consecutive lanes take nodes consecutive in
        // memory, along the layers for the slabs of the i axis, along i else
        const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
        int ad;
        long c1, c2;
        if (d == 0) {
            ad = (int)(t % (2 * G.g));
            c1 = (t / (2 * G.g)) % G.n[e1];
            c2 = (t / (2 * G.g)) / G.n[e1];
        } else {
            c1 = t % G.n[e1];
            ad = (int)((t / G.n[e1]) % (2 * G.g));
            c2 = (t / G.n[e1]) / (2 * G.g);
        }
        long off = G.base + (long)(ad < G.g ? ad - G.g : G.n[d] + ad - G.g) * G.sd[d] + c1 * G.sd[e1];
        if (ndim == 3) off += c2 * G.sd[e2];
        for (int v = 0; v < nvar; ++v) {
            const double x = gmem(src)[v * G.vol + off];
            gmem(dst1)[v * G.vol + off] = x;
            gmem(dst2)[v * G.vol + off] = x;
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
    const int* __restrict__ ord = kind_order(t_start, cap, BK_GHOST);
    int b = blockIdx.x < total ? find_block(st, nblk, blockIdx.x) : 0;
    for (long item = blockIdx.x; item < total; item += gridDim.x) {
        b = advance_block(st, nblk, b, item);
        const BBlock& B = t_blk[ord[b]];
        const long node = (item - st[b]) * 256 + threadIdx.x;
        if (node < frozen_slab_nodes(B.G, ndim))
            frozen_ghost_node(B.G, ndim, ndim + 2, B.q, B.A, B.B, node);
    }
}

// Interface exchange: for every link, the g ghost layers of block a on its
// side are copied from the interior layers of block b next to the opposite
// side.  which = 0, 1, 2: the state registers of RK stage 1 (q), 2 (A),
// 3 (B); which = 3: the metric arrays.  Node t of all links' ghost slabs
// (prefix sums lstart) per thread, its link found by binary search.  Within
// a slab consecutive lanes take nodes consecutive in memory: along the layer
// for a face of the i axis, along i for the other faces.
__global__ __launch_bounds__(256) void kb_halo(const int* __restrict__ t_nlink,
                                               const long* __restrict__ t_lstart,
                                               const LinkK* __restrict__ t_links,
                                               const BBlock* __restrict__ t_blk, int ndim, int which) {
    const int nl = *t_nlink;
    const long total = t_lstart[nl];
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        // the link of node t: the last li with lstart[li] <= t (binary search)
        int li = 0, hi = nl - 1;
        while (li < hi) {
            const int mid = (li + hi + 1) >> 1;
            if (t_lstart[mid] <= t)
                li = mid;
            else
                hi = mid - 1;
        }
        const LinkK L = t_links[li];
        const BBlock& A = t_blk[L.a];
        const BBlock& B = t_blk[L.b];
        const int g = A.G.g;
        // the transverse axes e1 < e2 (e2 = 2 only in 3D), then the node's
        // layer l and transverse indices c1, c2
        const int e1 = L.axis == 0 ? 1 : 0, e2 = L.axis == 2 ? 1 : 2;
        const long u = t - t_lstart[li];
        long c1, c2;
        int l;
        if (L.axis == 0) {
            l = (int)(u % g);
            c1 = (u / g) % A.G.n[e1];
            c2 = (u / g) / A.G.n[e1];
        } else {
            c1 = u % A.G.n[e1];
            l = (int)((u / A.G.n[e1]) % g);
            c2 = (u / A.G.n[e1]) / g;
        }
        long oa = A.G.base + c1 * A.G.sd[e1], ob = B.G.base + c1 * B.G.sd[e1];
        if (ndim == 3) {
            oa += c2 * A.G.sd[e2];
            ob += c2 * B.G.sd[e2];
        }
        const int ia = L.side ? A.G.n[L.axis] + l : -1 - l;
        const int ib = L.side ? l : B.G.n[L.axis] - 1 - l;
        oa += (long)ia * A.G.sd[L.axis];
        ob += (long)ib * B.G.sd[L.axis];
        if (which == 3) {
            gdouble* dst = gmem(const_cast<double*>(A.met));
            const int nmet = ndim == 3 ? 10 : 5;
            for (int v = 0; v < nmet; ++v) dst[v * A.G.vol + oa] = gmem(B.met)[v * B.G.vol + ob];
        } else {
            gdouble* dst = gmem(which == 0 ? A.q : (which == 1 ? A.A : A.B));
            const gdouble* src = gmem(which == 0 ? B.q : (which == 1 ? B.A : B.B));
            for (int v = 0; v < ndim + 2; ++v) dst[v * A.G.vol + oa] = src[v * B.G.vol + ob];
        }
    }
}

// ---------------------------------------------------------------------------
// boundary faces
// ---------------------------------------------------------------------------

struct BcK {
    int kind[3][2];  // 0 hold, 1 extrapolate, 2 slip wall, 3 moving planar shock
    const unsigned char* mask[3][2];
    const double* nodes;
    double pre[5], post[5];
    double normal[3];
    double offset, speed;
};

// ghost nodes (boundary nodes x layers) of face (a, side)
__device__ __host__ __forceinline__ long bc_face_nodes(const GeoK& G, int a) {
    const int e1 = a == 0 ? 1 : 0, e2 = a == 2 ? 1 : 2;
    return (long)G.n[e1] * G.n[e2] * G.g;
}

// Ghost node tt (boundary node fastest, then layer l = 1..g) of face
// (a, side) at time t: extrapolation copies the boundary node; the slip wall
// takes the mirror node l (from the boundary) with the momentum's component
// along the boundary node's unit metric vector of axis a reversed; the shock
// sets post or pre by the side of the moving plane. Masked nodes are left.
template <int DIM>
__device__ void apply_bc_node(const GeoK& G, const BcK& bc, int a, int side, const double* __restrict__ met,
                              double* __restrict__ q, double t, long tt) {
    constexpr int NV = DIM + 2, E = NV - 1;
    const int e1 = a == 0 ? 1 : 0, e2 = a == 2 ? 1 : 2;
    const long n1 = G.n[e1];
    const int g = G.g, kind = bc.kind[a][side], nb = G.n[a];
    const unsigned char* mask = bc.mask[a][side];
    const long sa = G.sd[a];
    const long i1 = tt % n1, r = tt / n1;
    const int l = (int)(r % g) + 1;
    const long i2 = r / g;
    if (mask && !mask[i2 * n1 + i1]) return;
    const long line = G.base + i1 * G.sd[e1] + i2 * G.sd[e2];
    const long og = line + (long)(side ? nb - 1 + l : -l) * sa;
    double Q[NV];
    if (kind == 1) {
        const long os = line + (long)(side ? nb - 1 : 0) * sa;
#pragma unroll
        for (int v = 0; v < NV; ++v) Q[v] = q[v * G.vol + os];
    } else if (kind == 2) {
        const long ob = line + (long)(side ? nb - 1 : 0) * sa;
        double nw[DIM], nn = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            nw[c] = met[(a * DIM + c) * G.vol + ob];
            nn += nw[c] * nw[c];
        }
        nn = sqrt(nn);
#pragma unroll
        for (int c = 0; c < DIM; ++c) nw[c] /= nn;
        const long os = line + (long)(side ? nb - 1 - l : l) * sa;
        double un = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) un += nw[c] * q[(1 + c) * G.vol + os];
        Q[0] = q[os];
#pragma unroll
        for (int c = 0; c < DIM; ++c) Q[1 + c] = q[(1 + c) * G.vol + os] - 2.0 * un * nw[c];
        Q[E] = q[E * G.vol + os];
    } else {
        double xn = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) xn += bc.normal[c] * bc.nodes[c * G.vol + og];
        const bool behind = xn < bc.offset + bc.speed * t;
#pragma unroll
        for (int v = 0; v < NV; ++v) Q[v] = behind ? bc.post[v] : bc.pre[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v * G.vol + og] = Q[v];
}

// The ghost layers of every face whose kind is not hold, in one launch at
// time t (or *tdev + t when the time lives on the device, as in a captured
// step): the ghost nodes of those faces (axis-major, low side first) are
// numbered one after another, one thread per ghost node.
template <int DIM>
__global__ __launch_bounds__(256) void k_bc_face(GeoK G, BcK bc, const double* __restrict__ met,
                                                  double* __restrict__ q, double t,
                                                  const double* __restrict__ tdev) {
    if (tdev) t += *tdev;
    long total = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int side = 0; side < 2; ++side)
            if (bc.kind[a][side]) total += bc_face_nodes(G, a);
    for (long u = (long)blockIdx.x * blockDim.x + threadIdx.x; u < total; u += (long)gridDim.x * blockDim.x) {
        // the face of ghost node u
        int a = 0, side = 0;
        long tt = u;
        for (int fi = 0; fi < 2 * DIM; ++fi) {
            const int fa = fi >> 1, fs = fi & 1;
            if (!bc.kind[fa][fs]) continue;
            const long cnt = bc_face_nodes(G, fa);
            if (tt < cnt) {
                a = fa;
                side = fs;
                break;
            }
            tt -= cnt;
        }
        apply_bc_node<DIM>(G, bc, a, side, met, q, t, tt);
    }
}

// The time of a captured step sequence, T = {t, t0, steps}: set before the
// replays; at the end of every step steps += 1 and t = t0 + steps dt (the
// step start times of an uncaptured run, without accumulated rounding).
__global__ void k_time_set(double* T, double t0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        T[0] = t0;
        T[1] = t0;
        T[2] = 0.0;
    }
}
__global__ void k_time_advance(double* T, double dt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double n = T[2] + 1.0;
        T[2] = n;
        T[0] = T[1] + n * dt;
    }
}

// ---------------------------------------------------------------------------
// viscous fluxes (periodic axes): node fluxes, then their central difference
// ---------------------------------------------------------------------------

// XCD-aware workgroup order: the dispatcher hands workgroups to the 8 XCDs
// round-robin (b -> XCD b mod 8), each XCD with its own L2.  Renumbering
// gives XCD x a contiguous range of the work instead of every eighth item.
__device__ __forceinline__ long xcd_block(long b, long nb) {
    const long per = nb / 8, rem = nb % 8, x = b % 8;
    return x * per + (x < rem ? x : rem) + b / 8;
}

// The node of this thread in the viscous kernels: a workgroup of 256 takes
// 64 (i) x 4 (j) nodes of one plane k.  The grid is cut into pencils of
// 64 x 32 nodes along k; within a pencil the workgroups run through its
// eight row groups fastest, then k, and each XCD takes a contiguous range of
// pencils (xcd_block).  A node's neighbours along the second and third axes
// then lie in the rows and planes its XCD read moments before (about 0.7 MB
// of L2 back): in plane order, every such neighbour three planes away was an
// L2 miss, and with one 64 x 4 column per k-run the row neighbours were.
constexpr int kViscRows = 4, kViscPencil = 8;  // rows per workgroup, row groups per pencil
__device__ __forceinline__ bool visc_node(const GeoK& G, int (&idx)[3]) {
    const unsigned L = (unsigned)xcd_block(blockIdx.x, gridDim.x);
    const unsigned nk = (unsigned)G.n[2], nit = ((unsigned)G.n[0] + 63u) / 64u;
    const unsigned r = L / kViscPencil, r2 = r / nk;
    idx[2] = (int)(r % nk);
    idx[0] = (int)((r2 % nit) * 64u + (threadIdx.x & 63u));
    idx[1] = (int)(((r2 / nit) * kViscPencil + L % kViscPencil) * kViscRows + (threadIdx.x >> 6));
    return idx[0] < G.n[0] && idx[1] < G.n[1];
}
inline long visc_blocks(const int n[3]) {
    const int pj = kViscRows * kViscPencil;
    return (long)((n[0] + 63) / 64) * ((n[1] + pj - 1) / pj) * kViscPencil * n[2];
}

// sixth-order central first derivative, offsets 1..3 (antisymmetric)
__device__ __forceinline__ double d6w(int o) { return o == 1 ? 45.0 / 60.0 : (o == 2 ? -9.0 / 60.0 : 1.0 / 60.0); }

// interior node `off` shifted by s along axis d with the periodic wrap
__device__ __forceinline__ long wrap_node(const GeoK& G, long off, int idx, int d, int s) {
    int t = idx + s;
    t = t < 0 ? t + G.n[d] : (t >= G.n[d] ? t - G.n[d] : t);
    return off + (long)(t - idx) * G.sd[d];
}

// primitives (u_1 .. u_DIM, T = p / rho) of node o
template <int DIM>
__device__ __forceinline__ void visc_prim(const double* __restrict__ q, long vol, long o, double gm1,
                                          double (&w)[DIM + 1]) {
    const double rho = q[o];
    const double ir = 1.0 / rho;
    double k2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double m = q[(1 + c) * vol + o];
        w[c] = m * ir;
        k2 += m * w[c];
    }
    w[DIM] = gm1 * (q[(DIM + 1) * vol + o] - 0.5 * k2) * ir;
}

// The contravariant viscous fluxes at node o from the sixth-order
// differences dphi[d][a] = D6_d(phi_a) of the primitives phi = (u, T) along
// every direction and the node's own primitives w: gradients by the chain
// rule dphi/dx_j = (1/V) sum_d s_{d,j} D6_d(phi), tau_ij = mu (du_i/dx_j +
// du_j/dx_i - 2/3 delta_ij div u), the physical fluxes (tau_1j .. tau_nj,
// u_i tau_ij + kappa dT/dx_j) and Fv~_d = sum_j s_{d,j} Fv_j.  fv: [DIM
// directions][DIM + 1 components] arrays in the state layout (the mass
// component, zero, is not stored).
template <int DIM>
__device__ __forceinline__ void visc_node_fluxes(const GeoK& G, double mu, double kappa,
                                                 const double* __restrict__ met, long o,
                                                 const double (&dphi)[DIM][DIM + 1], const double (&w)[DIM + 1],
                                                 double* __restrict__ fv) {
    constexpr int NP = DIM + 1, NMET = DIM == 3 ? 10 : 5;
    const double iV = 1.0 / met[(NMET - 1) * G.vol + o];
    double grad[NP][DIM];
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
        for (int j = 0; j < DIM; ++j) grad[a][j] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            const double sdj = met[(d * DIM + j) * G.vol + o] * iV;
#pragma unroll
            for (int a = 0; a < NP; ++a) grad[a][j] += sdj * dphi[d][a];
        }
    double div = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) div += grad[c][c];
    double F[DIM][NP];  // physical fluxes Fv_j, components 1..DIM+1
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        double work = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double tau = mu * (grad[a][j] + grad[j][a] - (a == j ? 2.0 / 3.0 * div : 0.0));
            F[j][a] = tau;
            work += w[a] * tau;
        }
        F[j][DIM] = work + kappa * grad[DIM][j];
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int v = 0; v < NP; ++v) {
            double sum = 0.0;
#pragma unroll
            for (int j = 0; j < DIM; ++j) sum += met[(d * DIM + j) * G.vol + o] * F[j][v];
            fv[(d * NP + v) * G.vol + o] = sum;
        }
}

// The viscous node fluxes of a 2D block, one lane per node: the primitives
// of the stencil neighbours are gathered along each direction.
template <int DIM>
__global__ __launch_bounds__(256) void k_visc_flux(GeoK G, double gamma, double mu, double kappa,
                                                    const double* __restrict__ met,
                                                    const double* __restrict__ q, double* __restrict__ fv) {
    constexpr int NP = DIM + 1;
    int idx[3];
    if (!visc_node(G, idx)) return;
    const long o = G.base + idx[0] + idx[1] * G.sd[1] + (long)idx[2] * G.sd[2];
    const double gm1 = gamma - 1.0;
    double dphi[DIM][NP];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
        for (int a = 0; a < NP; ++a) dphi[d][a] = 0.0;
#pragma unroll
        for (int s = 1; s <= 3; ++s) {
            double wp[NP], wm[NP];
            visc_prim<DIM>(q, G.vol, wrap_node(G, o, idx[d], d, s), gm1, wp);
            visc_prim<DIM>(q, G.vol, wrap_node(G, o, idx[d], d, -s), gm1, wm);
#pragma unroll
            for (int a = 0; a < NP; ++a) dphi[d][a] += d6w(s) * (wp[a] - wm[a]);
        }
    }
    double w[NP];
    visc_prim<DIM>(q, G.vol, o, gm1, w);
    visc_node_fluxes<DIM>(G, mu, kappa, met, o, dphi, w, fv);
}

// R = sum_d D6_d(Fv~_d) at every interior node of a 2D block (the mass
// component 0), one lane per node: the viscous part of the residual
// accumulator, before the inviscid sweeps subtract their flux differences.
template <int DIM>
__global__ __launch_bounds__(256) void k_visc_div(GeoK G, const double* __restrict__ fv, double* __restrict__ R) {
    constexpr int NP = DIM + 1;
    int idx[3];
    if (!visc_node(G, idx)) return;
    const long o = G.base + idx[0] + idx[1] * G.sd[1] + (long)idx[2] * G.sd[2];
    double acc[NP];
#pragma unroll
    for (int v = 0; v < NP; ++v) acc[v] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int s = 1; s <= 3; ++s) {
            const long op = wrap_node(G, o, idx[d], d, s), om = wrap_node(G, o, idx[d], d, -s);
#pragma unroll
            for (int v = 0; v < NP; ++v)
                acc[v] += d6w(s) * (fv[(d * NP + v) * G.vol + op] - fv[(d * NP + v) * G.vol + om]);
        }
    R[o] = 0.0;
#pragma unroll
    for (int v = 0; v < NP; ++v) R[(1 + v) * G.vol + o] = acc[v];
}

// 3D blocks: a workgroup (one lane per column) owns a kVmI (i) x kVmJ (j)
// tile of columns and a run of kVmK planes, and marches along k.  Each lane keeps the seven planes
// k-3 .. k+3 of its own column in registers (the zeta differences) and per
// plane the tile with a halo of three nodes in i and j is staged in LDS (the
// xi and eta differences): per node about 15 loads of q instead of 95, and
// every plane is read once per tile.  All axes are periodic, so every index
// wraps; lanes past the grid's edge load wrapped nodes and store nothing.
constexpr int kVmI = 64, kVmJ = 8, kVmK = 32, kVmHI = kVmI + 6, kVmHJ = kVmJ + 6;
inline long visc_march_blocks(const int n[3]) {
    return (long)((n[0] + kVmI - 1) / kVmI) * ((n[1] + kVmJ - 1) / kVmJ) * ((n[2] + kVmK - 1) / kVmK);
}
struct VmTile {
    int i0, j0, k0, k1;  // tile origin, planes [k0, k1)
    int i, j;            // this lane's column (wrapped into the grid)
    bool mine;           // the column is a node of the grid
};
__device__ __forceinline__ int wrapi(int t, int n) { return t < 0 ? t + n : (t >= n ? t - n : t); }
__device__ __forceinline__ VmTile vm_tile(const GeoK& G) {
    const unsigned L = (unsigned)xcd_block(blockIdx.x, gridDim.x);
    const unsigned nit = ((unsigned)G.n[0] + kVmI - 1) / kVmI, njt = ((unsigned)G.n[1] + kVmJ - 1) / kVmJ;
    VmTile t;
    t.i0 = (int)(L % nit) * kVmI;
    t.j0 = (int)((L / nit) % njt) * kVmJ;
    t.k0 = (int)(L / (nit * njt)) * kVmK;
    t.k1 = min(t.k0 + kVmK, G.n[2]);
    const int i = t.i0 + (int)(threadIdx.x % kVmI), j = t.j0 + (int)(threadIdx.x / kVmI);
    t.mine = i < G.n[0] && j < G.n[1];
    t.i = i % G.n[0];
    t.j = j % G.n[1];
    return t;
}
__device__ __forceinline__ long vm_off(const GeoK& G, int i, int j, int k) {
    return G.base + i + (long)j * G.sd[1] + (long)k * G.sd[2];
}

__global__ __launch_bounds__(kVmI * kVmJ) void k_visc_flux3(GeoK G, double gamma, double mu, double kappa,
                                                     const double* __restrict__ met,
                                                     const double* __restrict__ q, double* __restrict__ fv) {
    __shared__ double L[4][kVmHJ][kVmHI];  // primitives of plane k, tile and halo
    const VmTile t = vm_tile(G);
    const double gm1 = gamma - 1.0;
    const int li = (int)(threadIdx.x % kVmI) + 3, lj = (int)(threadIdx.x / kVmI) + 3;
    double P[7][4];  // this column's primitives at planes k-3 .. k+3
#pragma unroll
    for (int r = 0; r < 6; ++r) visc_prim<3>(q, G.vol, vm_off(G, t.i, t.j, wrapi(t.k0 - 3 + r, G.n[2])), gm1, P[r]);
    for (int k = t.k0; k < t.k1; ++k) {
        visc_prim<3>(q, G.vol, vm_off(G, t.i, t.j, wrapi(k + 3, G.n[2])), gm1, P[6]);
        __syncthreads();  // the previous plane's reads are done
        for (int e = threadIdx.x; e < kVmHI * kVmHJ; e += blockDim.x) {
            const int hi = e % kVmHI, hj = e / kVmHI;
            double w[4];
            visc_prim<3>(q, G.vol,
                         vm_off(G, (t.i0 - 3 + hi + 2 * G.n[0]) % G.n[0], (t.j0 - 3 + hj + 2 * G.n[1]) % G.n[1], k),
                         gm1, w);
#pragma unroll
            for (int a = 0; a < 4; ++a) L[a][hj][hi] = w[a];
        }
        __syncthreads();
        double dphi[3][4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            dphi[0][a] = 0.0;
            dphi[1][a] = 0.0;
            dphi[2][a] = 0.0;
#pragma unroll
            for (int s = 1; s <= 3; ++s) {
                dphi[0][a] += d6w(s) * (L[a][lj][li + s] - L[a][lj][li - s]);
                dphi[1][a] += d6w(s) * (L[a][lj + s][li] - L[a][lj - s][li]);
                dphi[2][a] += d6w(s) * (P[3 + s][a] - P[3 - s][a]);
            }
        }
        if (t.mine) visc_node_fluxes<3>(G, mu, kappa, met, vm_off(G, t.i, t.j, k), dphi, P[3], fv);
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int a = 0; a < 4; ++a) P[r][a] = P[r + 1][a];
    }
}

__global__ __launch_bounds__(kVmI * kVmJ) void k_visc_div3(GeoK G, const double* __restrict__ fv, double* __restrict__ R) {
    __shared__ double Lx[4][kVmJ][kVmHI];  // Fv~_xi of plane k: tile rows, halo in i
    __shared__ double Ly[4][kVmHJ][kVmI];  // Fv~_eta of plane k: tile columns, halo in j
    const VmTile t = vm_tile(G);
    const int ti = (int)(threadIdx.x % kVmI), tj = (int)(threadIdx.x / kVmI);
    double Z[7][4];  // this column's Fv~_zeta at planes k-3 .. k+3
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const long off = vm_off(G, t.i, t.j, wrapi(t.k0 - 3 + r, G.n[2]));
#pragma unroll
        for (int v = 0; v < 4; ++v) Z[r][v] = fv[(8 + v) * G.vol + off];
    }
    for (int k = t.k0; k < t.k1; ++k) {
        {
            const long off = vm_off(G, t.i, t.j, wrapi(k + 3, G.n[2]));
#pragma unroll
            for (int v = 0; v < 4; ++v) Z[6][v] = fv[(8 + v) * G.vol + off];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kVmHI * kVmJ; e += blockDim.x) {
            const int hi = e % kVmHI, hj = e / kVmHI;
            const long off = vm_off(G, (t.i0 - 3 + hi + 2 * G.n[0]) % G.n[0], (t.j0 + hj) % G.n[1], k);
#pragma unroll
            for (int v = 0; v < 4; ++v) Lx[v][hj][hi] = fv[v * G.vol + off];
        }
        for (int e = threadIdx.x; e < kVmI * kVmHJ; e += blockDim.x) {
            const int hi = e % kVmI, hj = e / kVmI;
            const long off = vm_off(G, (t.i0 + hi) % G.n[0], (t.j0 - 3 + hj + 2 * G.n[1]) % G.n[1], k);
#pragma unroll
            for (int v = 0; v < 4; ++v) Ly[v][hj][hi] = fv[(4 + v) * G.vol + off];
        }
        __syncthreads();
        double acc[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            acc[v] = 0.0;
#pragma unroll
            for (int s = 1; s <= 3; ++s) acc[v] += d6w(s) * (Lx[v][tj][ti + 3 + s] - Lx[v][tj][ti + 3 - s]);
#pragma unroll
            for (int s = 1; s <= 3; ++s) acc[v] += d6w(s) * (Ly[v][tj + 3 + s][ti] - Ly[v][tj + 3 - s][ti]);
#pragma unroll
            for (int s = 1; s <= 3; ++s) acc[v] += d6w(s) * (Z[3 + s][v] - Z[3 - s][v]);
        }
        if (t.mine) {
            const long o = vm_off(G, t.i, t.j, k);
            R[o] = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) R[(1 + v) * G.vol + o] = acc[v];
        }
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) Z[r][v] = Z[r + 1][v];
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
