// fp_inst.hip -- instantiates the sweep and face-flux kernels for one
// (precision, reconstruction) pair, selected at compile time by FP_INST_PREC
// (0 = FP64, 1 = mixed FP32) and FP_INST_RECON (0 = WENO5-JS, 1 = linear
// upwind, 2 = WENO7-JS, 3 = WENOCU6).  The build compiles this file once per pair, in parallel.
#include "fp_kernels.hpp"

#if !defined(FP_INST_PREC) || !defined(FP_INST_RECON)
#error "FP_INST_PREC and FP_INST_RECON must be defined"
#endif

#define FP_CAT2(a, b) a##b
#define FP_CAT(a, b) FP_CAT2(a, b)
#define FP_SUFFIX FP_CAT(FP_CAT(_p, FP_INST_PREC), FP_CAT(_r, FP_INST_RECON))

namespace fpk {

namespace {

constexpr int P = FP_INST_PREC;
constexpr int R = FP_INST_RECON;

inline unsigned blocks_for(long threads, int per_block) {
    return (unsigned)((threads + per_block - 1) / per_block);
}

// the scheme constants of direction d's sweep (its global LF speeds)
inline SchemeK dir_sk(const SchemeK& sk, int d) {
    SchemeK k = sk;
    k.glf += kGlfDirStride * d;
    return k;
}

template <int DIM, int DIR, int Y, int MODE>
void launch_wg_mode(const SweepArgs& a, const EpiK& ep, hipStream_t s) {
    constexpr int OTH = DIR == 1 ? 2 : 1;
    const long lblocks = ((long)a.G.n[0] * a.G.n[OTH] + 63) / 64;
    hipLaunchKernelGGL((k_sweep_wg<DIM, DIR, R, Y, P, MODE>), dim3((unsigned)(lblocks * a.nseg[DIR])),
                       dim3(256), 0, s, a.G, dir_sk(a.sk, DIR), a.met, a.qs, ep, a.S[DIR]);
}

template <int DIM, int DIR, int Y>
void launch_wg(const SweepArgs& a, const EpiK& ep, hipStream_t s) {
    switch (ep.mode) {
    case EPI_FIRST: launch_wg_mode<DIM, DIR, Y, EPI_FIRST>(a, ep, s); break;
    case EPI_MID: launch_wg_mode<DIM, DIR, Y, EPI_MID>(a, ep, s); break;
    case EPI_LAST_RES: launch_wg_mode<DIM, DIR, Y, EPI_LAST_RES>(a, ep, s); break;
    default: launch_wg_mode<DIM, DIR, Y, EPI_LAST_RK>(a, ep, s); break;
    }
}

// global LF speeds of every direction from the stage input (when asked
// for), in one launch of at most 128 workgroups of 1024 per direction
template <int DIM, int Y>
void launch_glf(const SweepArgs& a, hipStream_t s) {
    unsigned long long* set = reinterpret_cast<unsigned long long*>(const_cast<double*>(a.sk.glf));
    unsigned long long* next = reinterpret_cast<unsigned long long*>(a.glf_next);
    long most = 0;
    for (int d = 0; d < DIM; ++d) {
        const long segs = (long)(a.G.n[d] + kGlfSeg) / kGlfSeg * a.G.n[0] * a.G.n[1] * a.G.n[2] / a.G.n[d];
        most = segs > most ? segs : most;
    }
    const long bpd = (most + 1023) / 1024 < 128 ? (most + 1023) / 1024 : 128;
    hipLaunchKernelGGL((k_glf<DIM, Y, R == 2 ? 3 : 2>), dim3((unsigned)(bpd * DIM)), dim3(1024), 0, s, a.G,
                       a.sk.gamma, a.met, a.qs, set, next, (int)bpd);
}

// resident workgroups of a kernel on the current device (queried once)
template <class K>
int resident(K* kern) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 512;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 512;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(kern), 256, 0) !=
            hipSuccess ||
        per < 1)
        per = 1;
    return per * cus;
}

template <int DIM, int Y, bool ACC>
void launch_x_mode(const SweepArgs& a, const EpiK& ep, hipStream_t s) {
    static const int res = resident(&k_sweep_x<DIM, R, Y, P, ACC>);
    const long items = sweep_x_items(a.G.n, x_entries(P, R, Y));
    const long wgs = (items + 3) / 4;
    hipLaunchKernelGGL((k_sweep_x<DIM, R, Y, P, ACC>), dim3((unsigned)(wgs < res ? wgs : res)), dim3(256), 0,
                       s, a.G, a.sk, a.met, a.qs, ep);
}

// the xi sweep writes the accumulator (FIRST), or adds to it after the
// viscous part or a caller's accumulation
template <int DIM, int Y>
void launch_x(const SweepArgs& a, const EpiK& ep, hipStream_t s) {
    if (ep.mode == EPI_FIRST)
        launch_x_mode<DIM, Y, false>(a, ep, s);
    else
        launch_x_mode<DIM, Y, true>(a, ep, s);
}

template <int DIM, int Y>
hipError_t run_stage(const SweepArgs& a, hipStream_t s) {
    if (a.glf) {
        launch_glf<DIM, Y>(a, s);
        probe_mark(a.probe, PK_GLF, s);
    }
    launch_x<DIM, Y>(a, a.ep_first, s);
    probe_mark(a.probe, PK_XI, s);
    if constexpr (DIM == 3) {
        launch_wg<3, 1, Y>(a, a.ep_mid, s);
        probe_mark(a.probe, PK_ETA, s);
        launch_wg<3, 2, Y>(a, a.ep_last, s);
        probe_mark(a.probe, PK_ZETA, s);
    } else {
        launch_wg<2, 1, Y>(a, a.ep_last, s);
        probe_mark(a.probe, PK_ETA, s);
    }
    return hipGetLastError();
}

template <int DIM, int Y>
hipError_t run_dir(const SweepArgs& a, int dir, const EpiK& ep, hipStream_t s) {
    if (dir == 0) {
        launch_x<DIM, Y>(a, ep, s);
    } else if (dir == 1) {
        launch_wg<DIM, 1, Y>(a, ep, s);
    } else if constexpr (DIM == 3) {
        launch_wg<3, 2, Y>(a, ep, s);
    }
    return hipGetLastError();
}

template <int DIM>
dir_fn pick_dir(int Y) {
    switch (Y) {
    case 2: return &run_dir<DIM, 2>;
    case 4: return &run_dir<DIM, 4>;
    case 6: return &run_dir<DIM, 6>;
    case 8: return &run_dir<DIM, 8>;
    }
    return nullptr;
}

template <int DIM, int DIR, int Y>
hipError_t run_faceflux(const GeoK& G, const SchemeK& sk, const double* met, const double* q,
                        double* out, hipStream_t s) {
    long total = 1;
    for (int d = 0; d < 3; ++d) total *= (long)G.n[d] + (d == DIR ? 1 : 0);
    hipLaunchKernelGGL((k_face_flux<DIM, DIR, R, Y, P>), dim3(blocks_for(total, 256)), dim3(256), 0,
                       s, G, sk, met, q, out);
    return hipGetLastError();
}

template <int DIM>
stage_fn pick_stage(int Y) {
    switch (Y) {
    case 2: return &run_stage<DIM, 2>;
    case 4: return &run_stage<DIM, 4>;
    case 6: return &run_stage<DIM, 6>;
    case 8: return &run_stage<DIM, 8>;
    }
    return nullptr;
}

template <int DIM, int DIR>
faceflux_fn pick_ff(int Y) {
    switch (Y) {
    case 2: return &run_faceflux<DIM, DIR, 2>;
    case 4: return &run_faceflux<DIM, DIR, 4>;
    case 6: return &run_faceflux<DIM, DIR, 6>;
    case 8: return &run_faceflux<DIM, DIR, 8>;
    }
    return nullptr;
}

template <int DIM, int Y>
hipError_t run_batch_stage(const BTab& t, const SchemeK& sk, int stage, const int grid[3], int only,
                           hipStream_t s) {
    if (only < 0 || only == BK_X)
        hipLaunchKernelGGL((kb_sweep_x<DIM, R, Y, P>), dim3(grid[0]), dim3(256), 0, s, t.nblk, t.start, t.blk,
                           t.cap, sk, stage);
    if (only < 0 || only == BK_ETA)
        hipLaunchKernelGGL((kb_sweep_wg<DIM, 1, R, Y, P>), dim3(grid[1]), dim3(256), 0, s, t.nblk, t.start,
                           t.blk, t.cap, sk, stage);
    if constexpr (DIM == 3)
        if (only < 0 || only == BK_ZETA)
            hipLaunchKernelGGL((kb_sweep_wg<3, 2, R, Y, P>), dim3(grid[2]), dim3(256), 0, s, t.nblk, t.start,
                               t.blk, t.cap, sk, stage);
    return hipGetLastError();
}

template <int DIM, int Y>
int batch_occ(int kind) {
    int nb = 0;
    hipError_t e = hipSuccess;
    if (kind == BK_X)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_sweep_x<DIM, R, Y, P>, 256, 0);
    else if (kind == BK_ETA || DIM == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_sweep_wg<DIM, 1, R, Y, P>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_sweep_wg<DIM, DIM - 1, R, Y, P>, 256, 0);
    return e == hipSuccess ? nb : 0;
}

template <int DIM>
batch_stage_fn pick_batch(int Y) {
    switch (Y) {
    case 2: return &run_batch_stage<DIM, 2>;
    case 4: return &run_batch_stage<DIM, 4>;
    case 6: return &run_batch_stage<DIM, 6>;
    case 8: return &run_batch_stage<DIM, 8>;
    }
    return nullptr;
}

template <int DIM>
batch_occ_fn pick_occ(int Y) {
    switch (Y) {
    case 2: return &batch_occ<DIM, 2>;
    case 4: return &batch_occ<DIM, 4>;
    case 6: return &batch_occ<DIM, 6>;
    case 8: return &batch_occ<DIM, 8>;
    }
    return nullptr;
}

}  // namespace

stage_fn FP_CAT(get_stage, FP_SUFFIX)(int ndim, int Y) {
    return ndim == 3 ? pick_stage<3>(Y) : pick_stage<2>(Y);
}

dir_fn FP_CAT(get_dir, FP_SUFFIX)(int ndim, int Y) {
    return ndim == 3 ? pick_dir<3>(Y) : pick_dir<2>(Y);
}

batch_stage_fn FP_CAT(get_batch_stage, FP_SUFFIX)(int ndim, int Y) {
    return ndim == 3 ? pick_batch<3>(Y) : pick_batch<2>(Y);
}

batch_occ_fn FP_CAT(get_batch_occ, FP_SUFFIX)(int ndim, int Y) {
    return ndim == 3 ? pick_occ<3>(Y) : pick_occ<2>(Y);
}

faceflux_fn FP_CAT(get_faceflux, FP_SUFFIX)(int ndim, int dir, int Y) {
    if (ndim == 3) {
        if (dir == 0) return pick_ff<3, 0>(Y);
        if (dir == 1) return pick_ff<3, 1>(Y);
        return pick_ff<3, 2>(Y);
    }
    if (dir == 0) return pick_ff<2, 0>(Y);
    return pick_ff<2, 1>(Y);
}

}  // namespace fpk
