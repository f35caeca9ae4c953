// fp_api.hip -- host side of the C ABI declared in include/fp.h: argument
// validation, launch geometry, the RK3 stage sequence and the step-graph
// cache of fp_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fp.h"
#include "fp_kernels.hpp"
#include "fp_util_kernels.hpp"

namespace fpk {

#define FP_DECL_GET(P, R)                                           \
    stage_fn get_stage_p##P##_r##R(int ndim, int Y);                \
    dir_fn get_dir_p##P##_r##R(int ndim, int Y);                    \
    batch_stage_fn get_batch_stage_p##P##_r##R(int ndim, int Y);    \
    batch_occ_fn get_batch_occ_p##P##_r##R(int ndim, int Y);        \
    faceflux_fn get_faceflux_p##P##_r##R(int ndim, int dir, int Y);
FP_DECL_GET(0, 0)
FP_DECL_GET(0, 1)
FP_DECL_GET(0, 2)
FP_DECL_GET(0, 3)
FP_DECL_GET(1, 0)
FP_DECL_GET(1, 1)
FP_DECL_GET(1, 2)
FP_DECL_GET(1, 3)
#undef FP_DECL_GET

// the instantiation of one (precision, reconstruction) pair
#define FP_PICK(name, prec, recon, ...)                                                        \
    ((prec) == 0 ? ((recon) == 0   ? name##_p0_r0(__VA_ARGS__)                                 \
                    : (recon) == 1 ? name##_p0_r1(__VA_ARGS__)                                 \
                    : (recon) == 2 ? name##_p0_r2(__VA_ARGS__)                                 \
                                   : name##_p0_r3(__VA_ARGS__))                                \
                 : ((recon) == 0   ? name##_p1_r0(__VA_ARGS__)                                 \
                    : (recon) == 1 ? name##_p1_r1(__VA_ARGS__)                                 \
                    : (recon) == 2 ? name##_p1_r2(__VA_ARGS__)                                 \
                                   : name##_p1_r3(__VA_ARGS__)))

stage_fn get_stage_fn(int ndim, int recon, int Y, int prec) {
    return FP_PICK(get_stage, prec, recon, ndim, Y);
}

dir_fn get_dir_fn(int ndim, int recon, int Y, int prec) {
    return FP_PICK(get_dir, prec, recon, ndim, Y);
}

batch_stage_fn get_batch_stage_fn(int ndim, int recon, int Y, int prec) {
    return FP_PICK(get_batch_stage, prec, recon, ndim, Y);
}

batch_occ_fn get_batch_occ_fn(int ndim, int recon, int Y, int prec) {
    return FP_PICK(get_batch_occ, prec, recon, ndim, Y);
}

faceflux_fn get_faceflux_fn(int ndim, int dir, int recon, int Y, int prec) {
    return FP_PICK(get_faceflux, prec, recon, ndim, dir, Y);
}
#undef FP_PICK

}  // namespace fpk

using namespace fpk;

namespace {

thread_local std::string g_err;

fp_status fail(fp_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

fp_status hip_fail(hipError_t e, const char* what) {
    return fail(FP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

fp_status check_grid(const fp_grid* g) {
    if (!g) return fail(FP_EINVAL, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(FP_EINVAL, "ndim must be 2 or 3 (got %d)", g->ndim);
    if (g->ghost < 3 || g->ghost > 8) return fail(FP_EINVAL, "ghost must be in [3, 8] (got %d)", g->ghost);
    for (int d = 0; d < g->ndim; ++d) {
        if (g->n[d] < 1) return fail(FP_EINVAL, "n[%d] must be >= 1", d);
        if (g->bc[d] != FP_BC_PERIODIC && g->bc[d] != FP_BC_FROZEN)
            return fail(FP_EINVAL, "bc[%d] must be FP_BC_PERIODIC or FP_BC_FROZEN", d);
        if (g->bc[d] == FP_BC_PERIODIC && g->n[d] < g->ghost)
            return fail(FP_EINVAL, "periodic axis %d needs n >= ghost (%d < %d)", d, g->n[d], g->ghost);
    }
    if (g->ndim == 2 && g->n[2] != 1) return fail(FP_EINVAL, "2D grids need n[2] == 1");
    long long tot = 1;
    for (int d = 0; d < g->ndim; ++d) tot *= (long long)(g->n[d] + 2 * g->ghost);
    // the kernels address one variable array with 32-bit byte offsets
    if (tot >= (1ll << 29)) return fail(FP_EINVAL, "grid too large: at most 2^29 nodes per block, ghosts included");
    return FP_OK;
}

fp_status check_scheme(const fp_grid* g, const fp_scheme* s) {
    if (!s) return fail(FP_EINVAL, "scheme is NULL");
    if (s->recon != FP_WENO5JS && s->recon != FP_LINUP5 && s->recon != FP_WENO7JS && s->recon != FP_WENOCU6)
        return fail(FP_EINVAL, "unknown recon %d", s->recon);
    const int Y = s->metric_order;
    if (Y != 2 && Y != 4 && Y != 6 && Y != 8)
        return fail(FP_EUNSUPPORTED, "metric_order must be 2, 4, 6 or 8 (got %d)", Y);
    if (g->ghost < Y / 2) return fail(FP_EINVAL, "metric_order %d needs ghost >= %d", Y, Y / 2);
    if (s->recon == FP_WENO7JS && g->ghost < 4) return fail(FP_EINVAL, "WENO7 needs ghost >= 4");
    if (s->reformulated != 0 && s->reformulated != 1) return fail(FP_EINVAL, "reformulated must be 0 or 1");
    if (s->precision != FP_FP64 && s->precision != FP_MIXED32)
        return fail(FP_EINVAL, "unknown precision %d", s->precision);
    if (!(s->gamma > 1.0)) return fail(FP_EINVAL, "gamma must exceed 1");
    if (!(s->weno_eps > 0.0)) return fail(FP_EINVAL, "weno_eps must be positive");
    if (s->splitting != FP_LLF && s->splitting != FP_GLF) return fail(FP_EINVAL, "unknown splitting %d", s->splitting);
    if (!(s->mu >= 0.0)) return fail(FP_EINVAL, "mu must be >= 0");
    if (s->mu > 0.0) {
        if (!(s->prandtl > 0.0)) return fail(FP_EINVAL, "prandtl must be positive");
        for (int d = 0; d < g->ndim; ++d)
            if (g->bc[d] != FP_BC_PERIODIC || g->n[d] < 7)
                return fail(FP_EUNSUPPORTED, "viscous fluxes need periodic axes of at least 7 nodes");
    }
    return FP_OK;
}

GeoK make_geo(const fp_grid* g) {
    GeoK G;
    const int nd = g->ndim;
    for (int d = 0; d < 3; ++d) {
        G.n[d] = d < nd ? g->n[d] : 1;
        G.bc[d] = d < nd ? g->bc[d] : FP_BC_FROZEN;
    }
    G.g = g->ghost;
    const long N0 = G.n[0] + 2L * G.g, N1 = G.n[1] + 2L * G.g;
    const long N2 = nd == 3 ? G.n[2] + 2L * G.g : 1;
    G.sd[0] = 1;
    G.sd[1] = N0;
    G.sd[2] = N0 * N1;
    G.vol = N0 * N1 * N2;
    G.base = G.g + G.g * N0 + (nd == 3 ? (long)G.g * N0 * N1 : 0);
    return G;
}

// The speed floor of local Lax-Friedrichs splitting: zeros in static device
// memory (zero-initialised, never written), its address fetched once per
// device with that device current.
__device__ double g_zero_speeds[3 * kGlfDirStride];
std::mutex g_zero_mu;
std::map<int, const double*> g_zero_ptr;

const double* zero_speeds() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_zero_mu);
    auto it = g_zero_ptr.find(dev);
    if (it != g_zero_ptr.end()) return it->second;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_zero_speeds)) != hipSuccess || !p) return nullptr;
    g_zero_ptr[dev] = static_cast<const double*>(p);
    return static_cast<const double*>(p);
}

SchemeK make_sk(const fp_scheme* s) {
    SchemeK k;
    k.gamma = s->gamma;
    k.eps = s->weno_eps;
    k.reform = s->reformulated;
    k.glf = nullptr;  // bound by bind_speeds once the arguments are checked
    return k;
}

// Segments of the eta / zeta sweeps.  A workgroup owns 64 lines and one
// segment of S nodes, evaluating S+1 faces four at a time.  The plan
// minimises (rounds of resident workgroups) x (iterations per workgroup),
// with two resident workgroups per CU on 256 CUs.
void plan_segments(const GeoK& G, int ndim, SweepArgs& a) {
    const long resident = 256L * 2;
    for (int d = 1; d < ndim; ++d) {
        const int oth = d == 1 ? 2 : 1;
        const long lblocks = ((long)G.n[0] * G.n[oth] + 63) / 64;
        const int nd = G.n[d];
        long best = -1;
        int bestS = nd;
        for (int ns = 1; ns <= nd; ++ns) {
            const int S = (nd + ns - 1) / ns;
            if (S < 4 && ns > 1) break;
            const long segs = (nd + S - 1) / S;
            const long iters = (S + 1 + 3) / 4;
            const long rounds = (lblocks * segs + resident - 1) / resident;
            const long cost = rounds * iters;
            if (best < 0 || cost < best) {
                best = cost;
                bestS = S;
            }
        }
        a.S[d] = bestS;
        a.nseg[d] = (nd + bestS - 1) / bestS;
    }
    a.S[0] = a.nseg[0] = 0;
    if (ndim == 2) a.S[2] = a.nseg[2] = 0;
}

struct Ctx {
    fp_grid grid;
    fp_scheme sch;
    GeoK G;
    SchemeK sk;
    stage_fn stage;
    size_t state_elems;
};

fp_status make_ctx(const fp_grid* g, const fp_scheme* s, Ctx& c) {
    fp_status st = check_grid(g);
    if (st) return st;
    st = check_scheme(g, s);
    if (st) return st;
    c.grid = *g;
    c.sch = *s;
    c.G = make_geo(g);
    c.sk = make_sk(s);
    c.stage = get_stage_fn(g->ndim, s->recon, s->metric_order, s->precision);
    if (!c.stage) return fail(FP_EUNSUPPORTED, "no kernel for this scheme");
    c.state_elems = (size_t)(g->ndim + 2) * c.G.vol;
    return FP_OK;
}

// the speed floor of the current device (after argument checks: it is the
// first HIP call of an entry point)
fp_status bind_speeds(SchemeK& k) {
    k.glf = zero_speeds();
    if (!k.glf) return fail(FP_EHIP, "device symbol of the speed floor not found");
    return FP_OK;
}

EpiK epi(int mode, double* R) {
    EpiK e;
    std::memset(&e, 0, sizeof e);
    e.mode = mode;
    e.R = R;
    return e;
}

// the viscous part of the residual accumulator: R = sum_d D6_d(Fv~_d) from
// the node fluxes of `qs` (written to vwork); the sweeps then accumulate
void launch_viscous(const Ctx& c, const double* met, const double* qs, double* vwork, double* R,
                    hipStream_t s, Probe* probe = nullptr) {
    const double gam = c.sch.gamma, mu = c.sch.mu;
    const double kappa = mu * gam / ((gam - 1.0) * c.sch.prandtl);
    if (c.grid.ndim == 3) {
        const dim3 grid((unsigned)visc_march_blocks(c.G.n));
        hipLaunchKernelGGL(k_visc_flux3, grid, dim3(kVmI * kVmJ), 0, s, c.G, gam, mu, kappa, met, qs, vwork);
        probe_mark(probe, PK_VFLUX, s);
        hipLaunchKernelGGL(k_visc_div3, grid, dim3(kVmI * kVmJ), 0, s, c.G, (const double*)vwork, R);
        probe_mark(probe, PK_VDIV, s);
    } else {
        const dim3 grid((unsigned)visc_blocks(c.G.n));
        hipLaunchKernelGGL(k_visc_flux<2>, grid, dim3(256), 0, s, c.G, gam, mu, kappa, met, qs, vwork);
        probe_mark(probe, PK_VFLUX, s);
        hipLaunchKernelGGL(k_visc_div<2>, grid, dim3(256), 0, s, c.G, (const double*)vwork, R);
        probe_mark(probe, PK_VDIV, s);
    }
}

// one residual evaluation; the last sweep applies `last`; with a viscous
// scheme the viscous part initialises R first
hipError_t run_residual(const Ctx& c, const double* met, const double* qs, double* R,
                        const EpiK& last, hipStream_t s, double* vwork = nullptr) {
    const bool visc = c.sch.mu > 0.0;
    if (visc) launch_viscous(c, met, qs, vwork, R, s);
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.G = c.G;
    a.sk = c.sk;
    a.met = met;
    a.qs = qs;
    a.ep_first = epi(visc ? EPI_MID : EPI_FIRST, R);
    a.ep_mid = epi(EPI_MID, R);
    a.ep_last = last;
    plan_segments(c.G, c.grid.ndim, a);
    return c.stage(a, s);
}

// the boundary faces of `qs` at time t: one launch over every face that is not held
void launch_bcs(const Ctx& c, const BcK& bc, const double* met, double* qs, double t, hipStream_t s,
                const double* tdev = nullptr, Probe* probe = nullptr) {
    long total = 0;
    for (int a = 0; a < c.grid.ndim; ++a)
        for (int side = 0; side < 2; ++side)
            if (bc.kind[a][side] != FP_FACE_HOLD) total += bc_face_nodes(c.G, a);
    if (total == 0) return;
    const long blocks = (total + 255) / 256;
    const dim3 grid((unsigned)(blocks < 2048 ? blocks : 2048));
    if (c.grid.ndim == 3)
        hipLaunchKernelGGL(k_bc_face<3>, grid, dim3(256), 0, s, c.G, bc, met, qs, t, tdev);
    else
        hipLaunchKernelGGL(k_bc_face<2>, grid, dim3(256), 0, s, c.G, bc, met, qs, t, tdev);
    probe_mark(probe, PK_BC, s);
}

// The workspace tail (after the three state-sized arrays): three sets of
// global LF speeds (RK stage k reduces into set k and zeroes set k + 1 mod 3
// for the next stage), then the device time of fp_solve_bcs.
constexpr size_t kGlfBytes = 2048;
// launches of one instrumented step, at most: run start (2) + 3 stages x
// (boundary faces, 2 viscous, speeds, 3 sweeps)
constexpr int kProfileMax = 32;
constexpr size_t kTimeSlot = 3 * kGlfSetStride;  // in doubles
static_assert((kTimeSlot + 3) * sizeof(double) <= kGlfBytes, "the workspace tail is too small");

// the frozen ghost slabs of q into the two stage registers (nothing in a
// step writes them again, so a run of steps needs this once)
void launch_frozen(const Ctx& c, const double* q, double* work, hipStream_t s, Probe* probe = nullptr) {
    bool frozen = false;
    for (int d = 0; d < c.grid.ndim; ++d) frozen = frozen || c.grid.bc[d] == FP_BC_FROZEN;
    if (!frozen) return;
    const long slab = frozen_slab_nodes(c.G, c.grid.ndim);
    hipLaunchKernelGGL(k_frozen_ghosts, dim3((unsigned)((slab + 255) / 256)), dim3(256), 0, s, c.G,
                       c.grid.ndim, c.grid.ndim + 2, q, work, work + c.state_elems);
    probe_mark(probe, PK_GHOST, s);
}

// what a run of RK steps needs once, before its first step: the frozen
// ghost layers of the stage registers, and (global LF speeds) the first
// stage's speed set zeroed
void launch_run_start(const Ctx& c, const double* q, double* work, hipStream_t s, Probe* probe = nullptr) {
    launch_frozen(c, q, work, s, probe);
    if (c.sch.splitting == FP_GLF) {
        hipLaunchKernelGGL(k_glf_reset<2>, dim3(1), dim3(64), 0, s,
                           reinterpret_cast<unsigned long long*>(work + 3 * c.state_elems));
        probe_mark(probe, PK_GLF_RESET, s);
    }
}

// One TVD RK3 step: q -> A -> B -> q with residual accumulator R; with
// `ghosts`, the run-start work (frozen ghost layers of q into A and B, the
// first speed set zeroed) comes first.  With boundary faces, each stage's
// input gets its ghost layers at the stage time t, t + dt, t + dt/2; with
// global LF speeds, stage k reduces into the workspace tail's set k.
// (tdev: the step's start time on the device, then the stage times are
// *tdev + (0, dt, dt/2) and `t` is ignored)
hipError_t run_rk3(const Ctx& c, const double* met, double* q, double* work, double dt, hipStream_t s,
                   const BcK* bc = nullptr, double t = 0.0, double* vwork = nullptr, bool ghosts = true,
                   const double* tdev = nullptr, Probe* probe = nullptr) {
    const bool visc = c.sch.mu > 0.0;
    double* A = work;
    double* B = work + c.state_elems;
    double* R = work + 2 * c.state_elems;
    const bool glf = c.sch.splitting == FP_GLF;
    double* sets = work + 3 * c.state_elems;
    const double t0 = tdev ? 0.0 : t;
    const double stage_t[3] = {t0, t0 + dt, t0 + 0.5 * dt};
    if (ghosts) launch_run_start(c, q, work, s, probe);
    const double* metV = met + (size_t)(c.grid.ndim == 3 ? 9 : 4) * c.G.vol;
    const double* in[3] = {q, A, B};
    double* out[3] = {A, B, q};
    const double ca[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    const double cb[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    for (int k = 0; k < 3; ++k) {
        if (bc) launch_bcs(c, *bc, met, const_cast<double*>(in[k]), stage_t[k], s, tdev, probe);
        if (visc) launch_viscous(c, met, in[k], vwork, R, s, probe);
        EpiK e = epi(EPI_LAST_RK, R);
        e.stage0 = k == 0;
        e.out = out[k];
        e.metV = metV;
        e.qin = in[k];
        e.qn = q;
        e.dt = dt;
        e.a = ca[k];
        e.b = cb[k];
        SweepArgs a;
        std::memset(&a, 0, sizeof a);
        a.G = c.G;
        a.sk = c.sk;
        if (glf) {
            a.sk.glf = sets + kGlfSetStride * k;
            a.glf_next = sets + kGlfSetStride * ((k + 1) % 3);
            a.glf = 1;
        }
        a.met = met;
        a.qs = in[k];
        a.probe = probe;
        a.ep_first = epi(visc ? EPI_MID : EPI_FIRST, R);
        a.ep_mid = epi(EPI_MID, R);
        a.ep_last = e;
        plan_segments(c.G, c.grid.ndim, a);
        hipError_t err = c.stage(a, s);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// ---- workspace of fp_rk3_step_noalloc ----

// Static device memory, one copy per GPU, held until the process ends.  In
// host code `scratch` names a host-side stand-in, never the device array:
// the device address is fetched per device with hipGetSymbolAddress and
// only that pointer is passed to kernels.
static __device__ __align__(256) double scratch[FP_NOALLOC_WORK_BYTES / sizeof(double)];
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;

// the device address of `scratch` on the current device (fetched on the
// first call on that device, with it current)
fp_status scratch_ptr(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return FP_OK;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (no-allocation workspace)");
    if (!p) return fail(FP_EHIP, "hipGetSymbolAddress returned NULL for the no-allocation workspace");
    g_scratch_ptr[dev] = static_cast<double*>(p);
    *out = static_cast<double*>(p);
    return FP_OK;
}

// ---- step graph cache of fp_solve ----

struct GraphKey {
    int dev;
    fp_grid g;
    fp_scheme s;
    const double* met;
    double* q;
    double* work;
    double dt;
    bool operator<(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) < 0; }
};

std::mutex g_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;

// step graphs of fp_solve_bcs: the key adds the boundary faces
struct BcGraphKey {
    GraphKey k;
    BcK bc;
    bool operator<(const BcGraphKey& o) const { return std::memcmp(this, &o, sizeof(BcGraphKey)) < 0; }
};
std::map<BcGraphKey, hipGraphExec_t> g_bc_graphs;

std::map<int, hipStream_t> g_capture_streams;

// the stream graphs are captured on, one per device (call with g_mu held)
hipError_t capture_stream(int dev, hipStream_t* cs) {
    auto sit = g_capture_streams.find(dev);
    if (sit != g_capture_streams.end()) {
        *cs = sit->second;
        return hipSuccess;
    }
    hipError_t e = hipStreamCreateWithFlags(cs, hipStreamNonBlocking);
    if (e == hipSuccess) g_capture_streams[dev] = *cs;
    return e;
}

// ---- batches ----

constexpr int kSegTargets[] = {15, 23, 31, 47, 63, 95, 127};
constexpr int kSegDefault = 31;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }


}  // namespace

struct fp_batch {
    int dev = 0;
    fp_scheme sch{};
    SchemeK sk{};
    int cap = 0;
    int seg[3] = {0, kSegDefault, kSegDefault};  // eta / zeta segment length targets
    size_t part_bytes = 0;  // one part's tables: [nblk | start | blocks]
    char* dmem = nullptr;   // device tables, part 0 = 2D blocks, part 1 = 3D blocks
    char* hstage = nullptr; // pinned host image of dmem
    hipEvent_t staged = nullptr;
    bool pending = false;   // a staging copy may still read hstage
    std::vector<fp_block> blocks;
    std::vector<fp_link> links;  // interfaces, as given (global block indices)
    int maxl = 0;                // link capacity per part (6 per block)
    int nblk[2] = {0, 0};
    BTab tab[2]{};
    const int* lnk_n[2] = {nullptr, nullptr};     // device: links per part
    const long* lnk_start[2] = {nullptr, nullptr}; // device: prefix sums of ghost-slab nodes
    const LinkK* lnk[2] = {nullptr, nullptr};     // device: the links
    int grid[2][BK_KINDS]{};
    batch_stage_fn fn[2] = {nullptr, nullptr};
    // step graphs by mask: bits 0/1 non-empty 2D/3D part, bits 2/3 that part has links
    hipGraphExec_t graph[16] = {};
    int nlink[2] = {0, 0};  // links per part (no exchange launches without)
    hipStream_t cs = nullptr;
    bool tuned_from_cache = false;  // the last autotune reused a cached choice
};

namespace {

// The autotuner's choices, per process: keyed by the scheme (reconstruction,
// precision, metric order) and a size class of the batch (which
// dimensionalities it holds, and per dimensionality the binary orders of
// magnitude of its node count and of its mean line lengths along eta and
// zeta).
struct TuneKey {
    int recon, prec, Y, mask;
    int cls[2][3];
    bool operator<(const TuneKey& o) const { return std::memcmp(this, &o, sizeof(TuneKey)) < 0; }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;

int ilog2(double x) { return x >= 1.0 ? (int)std::floor(std::log2(x)) : 0; }

TuneKey tune_key(const fp_batch* b) {
    TuneKey k;
    std::memset(&k, 0, sizeof k);
    k.recon = b->sch.recon;
    k.prec = b->sch.precision;
    k.Y = b->sch.metric_order;
    k.mask = (b->nblk[0] > 0 ? 1 : 0) | (b->nblk[1] > 0 ? 2 : 0);
    for (int p = 0; p < 2; ++p) {
        double nodes = 0.0, ne = 0.0, nz = 0.0;
        int cnt = 0;
        for (const fp_block& fb : b->blocks) {
            if (fb.grid.ndim != (p == 0 ? 2 : 3)) continue;
            nodes += (double)fb.grid.n[0] * fb.grid.n[1] * (fb.grid.ndim == 3 ? fb.grid.n[2] : 1);
            ne += fb.grid.n[1];
            nz += fb.grid.ndim == 3 ? fb.grid.n[2] : 0;
            ++cnt;
        }
        if (cnt == 0) continue;
        k.cls[p][0] = ilog2(nodes);
        k.cls[p][1] = ilog2(ne / cnt);
        k.cls[p][2] = ilog2(nz / cnt);
    }
    return k;
}

// part layout: [nblk | 256 B][start: BK_KINDS x (cap + 1) longs, then the
// kinds' block orders: BK_KINDS x cap ints][blocks: cap][links ...]
size_t start_offset() { return 256; }
size_t blk_offset(int cap) {
    return 256 + align256(sizeof(long) * BK_KINDS * (size_t)(cap + 1) + sizeof(int) * BK_KINDS * (size_t)cap);
}
// link region of a part: [nlink | 256 B][lstart: maxl + 1 longs][links: maxl]
size_t lnk_offset(int cap) { return align256(blk_offset(cap) + sizeof(BBlock) * (size_t)cap); }
size_t lnk_start_offset(int cap) { return lnk_offset(cap) + 256; }
size_t lnk_arr_offset(int cap, int maxl) {
    return lnk_start_offset(cap) + align256(sizeof(long) * (size_t)(maxl + 1));
}
size_t part_size(int cap, int maxl) { return align256(lnk_arr_offset(cap, maxl) + sizeof(LinkK) * (size_t)maxl); }

// ghost-slab nodes of a link: g layers times the other axes' interior extents
long link_nodes(const fp_grid& g, int axis) {
    long c = g.ghost;
    for (int e = 0; e < g.ndim; ++e)
        if (e != axis) c *= g.n[e];
    return c;
}

int seg_len(int nd, int target) {
    const int nseg = (nd + target - 1) / target;
    return (nd + nseg - 1) / nseg;
}

// Host image of the tables of both parts for `blocks` (already validated).
void build_tables(const fp_batch* b, const std::vector<fp_block>& blocks, const std::vector<fp_link>& links,
                  char* img, int nblk[2], int nlink[2]) {
    for (int p = 0; p < 2; ++p) {
        char* base = img + p * b->part_bytes;
        long* start = reinterpret_cast<long*>(base + start_offset());
        BBlock* blk = reinterpret_cast<BBlock*>(base + blk_offset(b->cap));
        int* ord = reinterpret_cast<int*>(start + BK_KINDS * (b->cap + 1));
        const int ndim = p == 0 ? 2 : 3;
        int n = 0;
        std::vector<std::array<long, BK_KINDS>> nitems;
        for (const fp_block& fb : blocks) {
            if (fb.grid.ndim != ndim) continue;
            BBlock& B = blk[n];
            std::memset(&B, 0, sizeof B);
            B.G = make_geo(&fb.grid);
            const size_t se = (size_t)(ndim + 2) * B.G.vol;
            B.met = fb.met;
            B.q = fb.q;
            B.A = fb.work;
            B.B = fb.work + se;
            B.R = fb.work + 2 * se;
            B.dt = fb.dt;
            B.S[0] = 0;
            B.S[1] = seg_len(B.G.n[1], b->seg[1]);
            B.S[2] = ndim == 3 ? seg_len(B.G.n[2], b->seg[2]) : 0;
            bool frozen = false;
            for (int d = 0; d < ndim; ++d) frozen = frozen || fb.grid.bc[d] == FP_BC_FROZEN;
            long items[BK_KINDS];
            items[BK_X] = sweep_x_items(B.G.n, x_entries(b->sch.precision, b->sch.recon, b->sch.metric_order));
            items[BK_ETA] = sweep_wg_items(B.G.n, 1, B.S[1]);
            items[BK_ZETA] = ndim == 3 ? sweep_wg_items(B.G.n, 2, B.S[2]) : 0;
            items[BK_GHOST] = frozen ? (frozen_slab_nodes(B.G, ndim) + 255) / 256 : 0;
            nitems.push_back({items[0], items[1], items[2], items[3]});
            ++n;
        }
        // Work lists.  Items go to workgroups cyclically, so the eta / zeta
        // lists put the blocks with the most iterations per item (longest
        // segments) first: every round of items then has similar lengths and
        // the workgroups finish together.  The xi and ghost items are of one
        // size: block order.
        for (int k = 0; k < BK_KINDS; ++k) {
            std::vector<int> o(n);
            for (int i = 0; i < n; ++i) o[i] = i;
            if (k == BK_ETA || k == BK_ZETA) {
                const int d = k == BK_ETA ? 1 : 2;
                std::stable_sort(o.begin(), o.end(), [&](int a, int c) { return blk[a].S[d] > blk[c].S[d]; });
            }
            long acc = 0;
            for (int i = 0; i < n; ++i) {
                ord[k * b->cap + i] = o[i];
                start[k * (b->cap + 1) + i] = acc;
                acc += nitems[o[i]][k];
            }
            start[k * (b->cap + 1) + n] = acc;
        }
        *reinterpret_cast<int*>(base) = n;
        nblk[p] = n;
        // the part's links, with block indices local to the part
        long* lstart = reinterpret_cast<long*>(base + lnk_start_offset(b->cap));
        LinkK* lk = reinterpret_cast<LinkK*>(base + lnk_arr_offset(b->cap, b->maxl));
        std::vector<int> local(blocks.size(), -1);
        int c = 0;
        for (size_t i = 0; i < blocks.size(); ++i)
            if (blocks[i].grid.ndim == ndim) local[i] = c++;
        int nl = 0;
        long lacc = 0;
        for (const fp_link& L : links) {
            if (local[L.block] < 0) continue;
            lstart[nl] = lacc;
            lk[nl].a = local[L.block];
            lk[nl].b = local[L.nbr];
            lk[nl].axis = L.axis;
            lk[nl].side = L.side;
            lacc += link_nodes(blocks[L.block].grid, L.axis);
            ++nl;
        }
        lstart[nl] = lacc;
        *reinterpret_cast<int*>(base + lnk_offset(b->cap)) = nl;
        nlink[p] = nl;
    }
}

// Copy the tables of `blocks` to the device in stream order.
fp_status upload_tables(fp_batch* b, const std::vector<fp_block>& blocks, const std::vector<fp_link>& links,
                        hipStream_t s) {
    if (b->pending) {
        hipError_t e = hipEventSynchronize(b->staged);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        b->pending = false;
    }
    int nblk[2], nlink[2];
    build_tables(b, blocks, links, b->hstage, nblk, nlink);
    hipError_t e = hipMemcpyAsync(b->dmem, b->hstage, 2 * b->part_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (batch tables)");
    e = hipEventRecord(b->staged, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    b->pending = true;
    b->nblk[0] = nblk[0];
    b->nblk[1] = nblk[1];
    b->nlink[0] = nlink[0];
    b->nlink[1] = nlink[1];
    return FP_OK;
}

// the frozen ghost slabs of every block's q into its two stage registers
void run_batch_ghosts(const fp_batch* b, int mask, hipStream_t s) {
    for (int p = 0; p < 2; ++p)
        if (mask & (1 << p))
            hipLaunchKernelGGL(kb_frozen_ghosts, dim3(b->grid[p][BK_GHOST]), dim3(256), 0, s, b->tab[p].nblk,
                               b->tab[p].start, b->tab[p].blk, b->tab[p].cap, p == 0 ? 2 : 3);
}

// One RK3 step of every block (with the ghost copy first when `ghosts`).
// Nothing in a step writes the stage registers' frozen ghost slabs (the
// sweeps write interiors; the interface exchange rewrites its own slabs
// before every stage), so a run of steps needs the copy only once.
hipError_t run_batch_step(const fp_batch* b, int mask, hipStream_t s, bool ghosts = true) {
    for (int p = 0; p < 2; ++p) {
        if (!(mask & (1 << p))) continue;
        const int ndim = p == 0 ? 2 : 3;
        if (ghosts)
            hipLaunchKernelGGL(kb_frozen_ghosts, dim3(b->grid[p][BK_GHOST]), dim3(256), 0, s, b->tab[p].nblk,
                               b->tab[p].start, b->tab[p].blk, b->tab[p].cap, ndim);
        for (int k = 0; k < 3; ++k) {
            if (mask & (4 << p))
                hipLaunchKernelGGL(kb_halo, dim3(b->grid[p][BK_GHOST]), dim3(256), 0, s, b->lnk_n[p],
                                   b->lnk_start[p], b->lnk[p], b->tab[p].blk, ndim, k);
            hipError_t e = b->fn[p](b->tab[p], b->sk, k, b->grid[p], -1, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

int batch_mask(const fp_batch* b) {
    return (b->nblk[0] > 0 ? 1 : 0) | (b->nblk[1] > 0 ? 2 : 0) | (b->nlink[0] > 0 ? 4 : 0) | (b->nlink[1] > 0 ? 8 : 0);
}

fp_status check_batch(const fp_batch* b) {
    if (!b) return fail(FP_EINVAL, "batch is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != b->dev) return fail(FP_EINVAL, "batch was created on device %d, current device is %d", b->dev, dev);
    return FP_OK;
}

}  // namespace

extern "C" {

size_t fp_state_bytes(const fp_grid* g) {
    if (check_grid(g)) return 0;
    return sizeof(double) * (size_t)(g->ndim + 2) * make_geo(g).vol;
}

size_t fp_metric_bytes(const fp_grid* g) {
    if (check_grid(g)) return 0;
    return sizeof(double) * (size_t)(g->ndim == 3 ? 10 : 5) * make_geo(g).vol;
}

size_t fp_coord_bytes(const fp_grid* g, int32_t Y) {
    if (check_grid(g) || (Y != 2 && Y != 4 && Y != 6 && Y != 8)) return 0;
    size_t tot = g->ndim;
    for (int d = 0; d < g->ndim; ++d) tot *= (size_t)(g->n[d] + 2 * (g->ghost + Y / 2));
    return sizeof(double) * tot;
}

size_t fp_work_bytes(const fp_grid* g) {
    if (check_grid(g)) return 0;
    return 3 * fp_state_bytes(g) + kGlfBytes;
}

const char* fp_last_error(void) { return g_err.c_str(); }

fp_status fp_metrics(const fp_grid* g, int32_t Y, const double* xyz, double* met, void* stream) {
    fp_status st = check_grid(g);
    if (st) return st;
    if (Y != 2 && Y != 4 && Y != 6 && Y != 8)
        return fail(FP_EUNSUPPORTED, "metric_order must be 2, 4, 6 or 8 (got %d)", Y);
    if (g->ghost < Y / 2) return fail(FP_EINVAL, "metric_order %d needs ghost >= %d", Y, Y / 2);
    if (!xyz || !met) return fail(FP_EINVAL, "NULL array");
    hipStream_t s = (hipStream_t)stream;
    const GeoK G = make_geo(g);
    CGeoK C;
    C.gc = g->ghost + Y / 2;
    long Nc[3];
    for (int d = 0; d < 3; ++d) Nc[d] = d < g->ndim ? g->n[d] + 2L * C.gc : 1;
    C.csd[0] = 1;
    C.csd[1] = Nc[0];
    C.csd[2] = Nc[0] * Nc[1];
    C.cvol = Nc[0] * Nc[1] * Nc[2];
    C.cbase = C.gc + C.gc * Nc[0] + (g->ndim == 3 ? (long)C.gc * Nc[0] * Nc[1] : 0);
    int lo[3], cnt[3];
    for (int d = 0; d < 3; ++d) {
        if (d >= g->ndim) {
            lo[d] = 0;
            cnt[d] = 1;
        } else if (g->bc[d] == FP_BC_PERIODIC) {
            lo[d] = 0;
            cnt[d] = g->n[d];
        } else {
            lo[d] = -g->ghost;
            cnt[d] = g->n[d] + 2 * g->ghost;
        }
    }
    const long tot = (long)cnt[0] * cnt[1] * cnt[2];
    const unsigned blocks = (unsigned)((tot + 127) / 128);
#define FP_MET_LAUNCH(D, YY) \
    hipLaunchKernelGGL((k_metrics<D, YY>), dim3(blocks), dim3(128), 0, s, G, C, xyz, met, lo[0], lo[1], lo[2], cnt[0], cnt[1], cnt[2])
    if (g->ndim == 3) {
        switch (Y) {
        case 2: FP_MET_LAUNCH(3, 2); break;
        case 4: FP_MET_LAUNCH(3, 4); break;
        case 6: FP_MET_LAUNCH(3, 6); break;
        default: FP_MET_LAUNCH(3, 8); break;
        }
    } else {
        switch (Y) {
        case 2: FP_MET_LAUNCH(2, 2); break;
        case 4: FP_MET_LAUNCH(2, 4); break;
        case 6: FP_MET_LAUNCH(2, 6); break;
        default: FP_MET_LAUNCH(2, 8); break;
        }
    }
#undef FP_MET_LAUNCH
    hipLaunchKernelGGL(k_periodic_fill, dim3((unsigned)((G.vol + 255) / 256)), dim3(256), 0, s, G,
                       g->ndim, g->ndim == 3 ? 10 : 5, met);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp_metrics launch");
    return FP_OK;
}

fp_status fp_face_fluxes(const fp_grid* g, const fp_scheme* sch, const double* met, const double* q,
                         int32_t dir, double* flux, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (sch->mu > 0.0) return fail(FP_EUNSUPPORTED, "viscous schemes take fp_viscous_residual / fp_solve_ns");
    if (sch->splitting == FP_GLF)
        return fail(FP_EUNSUPPORTED, "global LF speeds need the workspace of fp_rk3_step / fp_solve");
    if (dir < 0 || dir >= g->ndim) return fail(FP_EINVAL, "dir must be in [0, ndim)");
    if (!met || !q || !flux) return fail(FP_EINVAL, "NULL array");
    st = bind_speeds(c.sk);
    if (st) return st;
    faceflux_fn f = get_faceflux_fn(g->ndim, dir, sch->recon, sch->metric_order, sch->precision);
    if (!f) return fail(FP_EUNSUPPORTED, "no face-flux kernel for this scheme");
    hipError_t e = f(c.G, c.sk, met, q, flux, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fp_face_fluxes launch");
    return FP_OK;
}

fp_status fp_residual(const fp_grid* g, const fp_scheme* sch, const double* met, const double* q,
                      double* dqdt, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (sch->mu > 0.0) return fail(FP_EUNSUPPORTED, "viscous schemes take fp_viscous_residual / fp_solve_ns");
    if (sch->splitting == FP_GLF)
        return fail(FP_EUNSUPPORTED, "global LF speeds need the workspace of fp_rk3_step / fp_solve");
    if (!met || !q || !dqdt) return fail(FP_EINVAL, "NULL array");
    if ((const double*)dqdt == q) return fail(FP_EINVAL, "dqdt must not alias q");
    st = bind_speeds(c.sk);
    if (st) return st;
    EpiK last = epi(EPI_LAST_RES, dqdt);
    last.out = dqdt;
    last.metV = met + (size_t)(g->ndim == 3 ? 9 : 4) * c.G.vol;
    hipError_t e = run_residual(c, met, q, dqdt, last, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fp_residual launch");
    return FP_OK;
}

fp_status fp_residual_dir(const fp_grid* g, const fp_scheme* sch, const double* met, const double* q,
                          int32_t dir, double* acc, int32_t accumulate, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (sch->mu > 0.0) return fail(FP_EUNSUPPORTED, "viscous schemes take fp_viscous_residual / fp_solve_ns");
    if (sch->splitting == FP_GLF)
        return fail(FP_EUNSUPPORTED, "global LF speeds need the workspace of fp_rk3_step / fp_solve");
    if (dir < 0 || dir >= g->ndim) return fail(FP_EINVAL, "dir must be in [0, ndim)");
    if (accumulate != 0 && accumulate != 1) return fail(FP_EINVAL, "accumulate must be 0 or 1");
    if (!met || !q || !acc) return fail(FP_EINVAL, "NULL array");
    if ((const double*)acc == q) return fail(FP_EINVAL, "acc must not alias q");
    st = bind_speeds(c.sk);
    if (st) return st;
    dir_fn f = get_dir_fn(g->ndim, sch->recon, sch->metric_order, sch->precision);
    if (!f) return fail(FP_EUNSUPPORTED, "no sweep kernel for this scheme");
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.G = c.G;
    a.sk = c.sk;
    a.met = met;
    a.qs = q;
    plan_segments(c.G, g->ndim, a);
    hipError_t e = f(a, dir, epi(accumulate ? EPI_MID : EPI_FIRST, acc), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fp_residual_dir launch");
    return FP_OK;
}

fp_status fp_rk3_step(const fp_grid* g, const fp_scheme* sch, const double* met, double* q,
                      double* work, double dt, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (sch->mu > 0.0) return fail(FP_EUNSUPPORTED, "viscous schemes take fp_viscous_residual / fp_solve_ns");
    if (!met || !q || !work) return fail(FP_EINVAL, "NULL array");
    if (!(dt > 0.0)) return fail(FP_EINVAL, "dt must be positive");
    st = bind_speeds(c.sk);
    if (st) return st;
    hipError_t e = run_rk3(c, met, q, work, dt, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fp_rk3_step launch");
    return FP_OK;
}

fp_status fp_rk3_step_noalloc(const fp_grid* g, const fp_scheme* sch, const double* met, double* q, double dt,
                              void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (sch->mu > 0.0) return fail(FP_EUNSUPPORTED, "viscous schemes take fp_viscous_residual / fp_solve_ns");
    if (!met || !q) return fail(FP_EINVAL, "NULL array");
    if (!(dt > 0.0)) return fail(FP_EINVAL, "dt must be positive");
    const size_t need = fp_work_bytes(g);
    if (need > FP_NOALLOC_WORK_BYTES)
        return fail(FP_EINVAL, "grid needs %zu bytes of workspace; fp_rk3_step_noalloc holds %zu (use fp_rk3_step)",
                    need, (size_t)FP_NOALLOC_WORK_BYTES);
    st = bind_speeds(c.sk);
    if (st) return st;
    double* work = nullptr;
    st = scratch_ptr(&work);
    if (st) return st;
    hipError_t e = run_rk3(c, met, q, work, dt, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fp_rk3_step_noalloc launch");
    return FP_OK;
}

fp_status fp_solve(const fp_grid* g, const fp_scheme* sch, const double* met, double* q, double* work,
                   double dt, int64_t nsteps, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (sch->mu > 0.0) return fail(FP_EUNSUPPORTED, "viscous schemes take fp_viscous_residual / fp_solve_ns");
    if (!met || !q || !work) return fail(FP_EINVAL, "NULL array");
    if (!(dt > 0.0)) return fail(FP_EINVAL, "dt must be positive");
    if (nsteps < 0) return fail(FP_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return FP_OK;
    st = bind_speeds(c.sk);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    GraphKey key;
    std::memset(&key, 0, sizeof key);
    key.dev = dev;
    key.g = *g;
    key.s = *sch;
    key.met = met;
    key.q = q;
    key.work = work;
    key.dt = dt;
    hipGraphExec_t exec = nullptr;
    // held until the step graph's launches are enqueued: another thread may
    // evict and destroy cached graphs (a full cache, fp_release_cache)
    std::lock_guard<std::mutex> lk(g_mu);
    {
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) {
            exec = it->second;
        } else {
            hipStream_t cs;
            e = capture_stream(dev, &cs);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            hipError_t le = run_rk3(c, met, q, work, dt, cs, nullptr, 0.0, nullptr, false);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(cs, &graph);
            if (le != hipSuccess) {
                if (graph) hipGraphDestroy(graph);
                return hip_fail(le, "fp_solve capture");
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            if (g_graphs.size() >= 64) {
                for (auto& kv : g_graphs) hipGraphExecDestroy(kv.second);
                g_graphs.clear();
            }
            g_graphs[key] = exec;
        }
    }
    launch_run_start(c, q, work, s);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp_solve ghost copy");
    for (int64_t i = 0; i < nsteps; ++i) {
        e = hipGraphLaunch(exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    return FP_OK;
}

fp_status make_bck(const fp_grid* g, const fp_bcs* bcs, BcK& k) {
    if (!bcs) return fail(FP_EINVAL, "bcs is NULL");
    std::memset(&k, 0, sizeof k);
    for (int a = 0; a < 3; ++a)
        for (int side = 0; side < 2; ++side) {
            const int kind = bcs->kind[a][side];
            if (kind < FP_FACE_HOLD || kind > FP_FACE_SHOCK)
                return fail(FP_EINVAL, "face (%d, %d): unknown kind %d", a, side, kind);
            if (kind == FP_FACE_HOLD) continue;
            if (a >= g->ndim) return fail(FP_EINVAL, "face (%d, %d): no such axis", a, side);
            if (g->bc[a] != FP_BC_FROZEN)
                return fail(FP_EINVAL, "face (%d, %d): boundary faces need an FP_BC_FROZEN axis", a, side);
            if (kind == FP_FACE_WALL && g->n[a] < g->ghost + 1)
                return fail(FP_EINVAL, "face (%d, %d): a wall needs n > ghost along its axis", a, side);
            if (kind == FP_FACE_SHOCK && !bcs->nodes)
                return fail(FP_EINVAL, "face (%d, %d): the shock needs the node coordinates", a, side);
            k.kind[a][side] = kind;
            k.mask[a][side] = bcs->mask[a][side];
        }
    k.nodes = bcs->nodes;
    for (int v = 0; v < 5; ++v) {
        k.pre[v] = bcs->pre[v];
        k.post[v] = bcs->post[v];
    }
    for (int c = 0; c < 3; ++c) k.normal[c] = bcs->normal[c];
    k.offset = bcs->offset;
    k.speed = bcs->speed;
    return FP_OK;
}

fp_status fp_apply_bcs(const fp_grid* g, const fp_bcs* bcs, const double* met, double* q, double t,
                       void* stream) {
    fp_status st = check_grid(g);
    if (st) return st;
    if (!met || !q) return fail(FP_EINVAL, "NULL array");
    BcK k;
    st = make_bck(g, bcs, k);
    if (st) return st;
    Ctx c;
    c.grid = *g;
    c.G = make_geo(g);
    launch_bcs(c, k, met, q, t, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp_apply_bcs launch");
    return FP_OK;
}

fp_status fp_solve_bcs(const fp_grid* g, const fp_scheme* sch, const fp_bcs* bcs, const double* met,
                       double* q, double* work, double t0, double dt, int64_t nsteps, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (sch->mu > 0.0) return fail(FP_EUNSUPPORTED, "viscous schemes take fp_viscous_residual / fp_solve_ns");
    if (!met || !q || !work) return fail(FP_EINVAL, "NULL array");
    if (!(dt > 0.0)) return fail(FP_EINVAL, "dt must be positive");
    if (nsteps < 0) return fail(FP_EINVAL, "nsteps must be >= 0");
    BcK k;
    st = make_bck(g, bcs, k);
    if (st) return st;
    st = bind_speeds(c.sk);
    if (st) return st;
    if (nsteps == 0) return FP_OK;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    double* T = work + 3 * c.state_elems + kTimeSlot;  // {t, t0, steps}
    BcGraphKey key;
    std::memset(&key, 0, sizeof key);
    key.k.dev = dev;
    key.k.g = *g;
    key.k.s = *sch;
    key.k.met = met;
    key.k.q = q;
    key.k.work = work;
    key.k.dt = dt;
    key.bc = k;
    hipGraphExec_t exec = nullptr;
    // held until the step graph's launches are enqueued (as in fp_solve)
    std::lock_guard<std::mutex> lk(g_mu);
    {
        auto it = g_bc_graphs.find(key);
        if (it != g_bc_graphs.end()) {
            exec = it->second;
        } else {
            hipStream_t cs;
            e = capture_stream(dev, &cs);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            hipError_t le = run_rk3(c, met, q, work, dt, cs, &k, 0.0, nullptr, false, T);
            if (le == hipSuccess) {
                hipLaunchKernelGGL(k_time_advance, dim3(1), dim3(64), 0, cs, T, dt);
                le = hipGetLastError();
            }
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(cs, &graph);
            if (le != hipSuccess) {
                if (graph) hipGraphDestroy(graph);
                return hip_fail(le, "fp_solve_bcs capture");
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            if (g_bc_graphs.size() >= 64) {
                for (auto& kv : g_bc_graphs) hipGraphExecDestroy(kv.second);
                g_bc_graphs.clear();
            }
            g_bc_graphs[key] = exec;
        }
    }
    hipLaunchKernelGGL(k_time_set, dim3(1), dim3(64), 0, s, T, t0);
    launch_run_start(c, q, work, s);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp_solve_bcs launch");
    for (int64_t i = 0; i < nsteps; ++i) {
        e = hipGraphLaunch(exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    return FP_OK;
}

fp_status fp_profile_step(const fp_grid* g, const fp_scheme* sch, const fp_bcs* bcs, const double* met,
                          double* q, double* work, double* vwork, double t, double dt, float* kernel_ms,
                          int32_t* kernel_kind, int32_t max_kernels, int32_t* n_kernels, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (!met || !q || !work || (sch->mu > 0.0 && !vwork)) return fail(FP_EINVAL, "NULL array");
    if (!kernel_ms || !kernel_kind || !n_kernels) return fail(FP_EINVAL, "NULL output");
    if (max_kernels < kProfileMax) return fail(FP_EINVAL, "max_kernels must be >= %d", kProfileMax);
    if (!(dt > 0.0)) return fail(FP_EINVAL, "dt must be positive");
    BcK k;
    if (bcs) {
        st = make_bck(g, bcs, k);
        if (st) return st;
    }
    st = bind_speeds(c.sk);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[kProfileMax + 1];
    hipError_t e = hipSuccess;
    int made = 0;
    while (made <= kProfileMax) {
        e = hipEventCreate(&ev[made]);
        if (e != hipSuccess) break;
        ++made;
    }
    Probe probe{ev, kernel_kind, 0, kProfileMax, hipSuccess};
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess)
        e = run_rk3(c, met, q, work, dt, s, bcs ? &k : nullptr, t, sch->mu > 0.0 ? vwork : nullptr, true,
                    nullptr, &probe);
    if (e == hipSuccess) e = probe.err;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess && probe.n > 0) e = hipEventSynchronize(ev[probe.n]);
    for (int i = 0; i < probe.n && e == hipSuccess; ++i) e = hipEventElapsedTime(&kernel_ms[i], ev[i], ev[i + 1]);
    for (int i = 0; i < made; ++i) hipEventDestroy(ev[i]);
    if (e != hipSuccess) return hip_fail(e, "fp_profile_step");
    *n_kernels = probe.n;
    return FP_OK;
}

size_t fp_viscous_work_bytes(const fp_grid* g) {
    if (check_grid(g)) return 0;
    return (size_t)g->ndim * (g->ndim + 1) * fp_state_bytes(g) / (g->ndim + 2);
}

fp_status fp_viscous_residual(const fp_grid* g, const fp_scheme* sch, const double* met, const double* q,
                              double* dqdt, double* vwork, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (sch->splitting == FP_GLF)
        return fail(FP_EUNSUPPORTED, "global LF speeds need the workspace of fp_solve_ns");
    if (!met || !q || !dqdt || (sch->mu > 0.0 && !vwork)) return fail(FP_EINVAL, "NULL array");
    if ((const double*)dqdt == q) return fail(FP_EINVAL, "dqdt must not alias q");
    st = bind_speeds(c.sk);
    if (st) return st;
    EpiK last = epi(EPI_LAST_RES, dqdt);
    last.out = dqdt;
    last.metV = met + (size_t)(g->ndim == 3 ? 9 : 4) * c.G.vol;
    hipError_t e = run_residual(c, met, q, dqdt, last, (hipStream_t)stream, vwork);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp_viscous_residual launch");
    return FP_OK;
}

fp_status fp_solve_ns(const fp_grid* g, const fp_scheme* sch, const double* met, double* q, double* work,
                      double* vwork, double dt, int64_t nsteps, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (!met || !q || !work || (sch->mu > 0.0 && !vwork)) return fail(FP_EINVAL, "NULL array");
    if (!(dt > 0.0)) return fail(FP_EINVAL, "dt must be positive");
    if (nsteps < 0) return fail(FP_EINVAL, "nsteps must be >= 0");
    st = bind_speeds(c.sk);
    if (st) return st;
    for (int64_t i = 0; i < nsteps; ++i) {
        hipError_t e = run_rk3(c, met, q, work, dt, (hipStream_t)stream, nullptr, 0.0, vwork);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "fp_solve_ns launch");
    }
    return FP_OK;
}

fp_status fp_max_dt(const fp_grid* g, const fp_scheme* sch, const double* met, const double* q,
                    double cfl, double* dt_dev, void* stream) {
    fp_status st = check_grid(g);
    if (st) return st;
    if (!sch || !(sch->gamma > 1.0)) return fail(FP_EINVAL, "bad scheme");
    if (!met || !q || !dt_dev) return fail(FP_EINVAL, "NULL array");
    if (!(cfl > 0.0)) return fail(FP_EINVAL, "cfl must be positive");
    hipStream_t s = (hipStream_t)stream;
    const GeoK G = make_geo(g);
    const long tot = (long)G.n[0] * G.n[1] * G.n[2];
    unsigned long long* bits = reinterpret_cast<unsigned long long*>(dt_dev);
    hipLaunchKernelGGL(k_dt_init, dim3(1), dim3(1), 0, s, bits);
    const unsigned blocks = (unsigned)((tot + 255) / 256);
    if (g->ndim == 3)
        hipLaunchKernelGGL(k_dt_reduce<3>, dim3(blocks), dim3(256), 0, s, G, sch->gamma, met, q, bits);
    else
        hipLaunchKernelGGL(k_dt_reduce<2>, dim3(blocks), dim3(256), 0, s, G, sch->gamma, met, q, bits);
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(1), 0, s, bits, cfl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp_max_dt launch");
    return FP_OK;
}

fp_status fp_check_state(const fp_grid* g, const fp_scheme* sch, const double* q, int32_t* flag_dev,
                         void* stream) {
    fp_status st = check_grid(g);
    if (st) return st;
    if (!sch || !(sch->gamma > 1.0)) return fail(FP_EINVAL, "bad scheme");
    if (!q || !flag_dev) return fail(FP_EINVAL, "NULL array");
    const GeoK G = make_geo(g);
    const long tot = (long)G.n[0] * G.n[1] * G.n[2];
    const unsigned blocks = (unsigned)((tot + 255) / 256);
    if (g->ndim == 3)
        hipLaunchKernelGGL(k_check_state<3>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, G,
                           sch->gamma, q, (int*)flag_dev);
    else
        hipLaunchKernelGGL(k_check_state<2>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, G,
                           sch->gamma, q, (int*)flag_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp_check_state launch");
    return FP_OK;
}

fp_status fp_batch_create(const fp_scheme* sch, int32_t max_blocks, fp_batch** out) {
    if (!out) return fail(FP_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_blocks < 1 || max_blocks > 65536) return fail(FP_EINVAL, "max_blocks must be in [1, 65536]");
    fp_grid g3{};
    g3.ndim = 3;
    g3.n[0] = g3.n[1] = g3.n[2] = 8;
    g3.ghost = sch ? ((sch->metric_order == 8 || sch->recon == FP_WENO7JS) ? 4 : 3) : 3;
    fp_status st = check_scheme(&g3, sch);
    if (st) return st;
    if (sch->splitting == FP_GLF) return fail(FP_EUNSUPPORTED, "batches use local LF speeds");
    if (sch->mu > 0.0) return fail(FP_EUNSUPPORTED, "batches are inviscid");
    fp_batch* b = new fp_batch();
    b->sch = *sch;
    b->sk = make_sk(sch);
    if (bind_speeds(b->sk) != FP_OK) {
        delete b;
        return FP_EHIP;
    }
    b->cap = max_blocks;
    b->maxl = 6 * max_blocks;
    b->part_bytes = part_size(max_blocks, b->maxl);
    hipError_t e = hipGetDevice(&b->dev);
    if (e == hipSuccess) e = hipMalloc((void**)&b->dmem, 2 * b->part_bytes);
    if (e != hipSuccess) {
        delete b;
        return fail(FP_ENOMEM, "batch tables: %s", hipGetErrorString(e));
    }
    e = hipHostMalloc((void**)&b->hstage, 2 * b->part_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        hipFree(b->dmem);
        delete b;
        return fail(FP_ENOMEM, "batch staging: %s", hipGetErrorString(e));
    }
    std::memset(b->hstage, 0, 2 * b->part_bytes);
    e = hipMemcpy(b->dmem, b->hstage, 2 * b->part_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->dev);
    if (e != hipSuccess) {
        fp_batch_destroy(b);
        return hip_fail(e, "fp_batch_create");
    }
    for (int p = 0; p < 2; ++p) {
        const int ndim = p == 0 ? 2 : 3;
        char* base = b->dmem + p * b->part_bytes;
        b->tab[p].nblk = reinterpret_cast<const int*>(base);
        b->tab[p].start = reinterpret_cast<const long*>(base + start_offset());
        b->tab[p].blk = reinterpret_cast<const BBlock*>(base + blk_offset(max_blocks));
        b->tab[p].cap = max_blocks;
        b->lnk_n[p] = reinterpret_cast<const int*>(base + lnk_offset(max_blocks));
        b->lnk_start[p] = reinterpret_cast<const long*>(base + lnk_start_offset(max_blocks));
        b->lnk[p] = reinterpret_cast<const LinkK*>(base + lnk_arr_offset(max_blocks, b->maxl));
        b->fn[p] = get_batch_stage_fn(ndim, sch->recon, sch->metric_order, sch->precision);
        batch_occ_fn occ = get_batch_occ_fn(ndim, sch->recon, sch->metric_order, sch->precision);
        if (!b->fn[p] || !occ) {
            fp_batch_destroy(b);
            return fail(FP_EUNSUPPORTED, "no batched kernel for this scheme");
        }
        for (int k = 0; k < 3; ++k) {
            const int per_cu = occ(k);
            b->grid[p][k] = (per_cu > 0 ? per_cu : 1) * cus;
        }
        b->grid[p][BK_GHOST] = 16 * cus;  // ghost copy and interface exchange: grid-stride, many nodes in flight
    }
    *out = b;
    return FP_OK;
}

fp_status fp_batch_set(fp_batch* b, const fp_block* blocks, int32_t nblocks, void* stream) {
    fp_status st = check_batch(b);
    if (st) return st;
    if (nblocks < 0 || nblocks > b->cap) return fail(FP_EINVAL, "nblocks must be in [0, %d]", b->cap);
    if (nblocks > 0 && !blocks) return fail(FP_EINVAL, "blocks is NULL");
    for (int i = 0; i < nblocks; ++i) {
        const fp_block& fb = blocks[i];
        st = check_grid(&fb.grid);
        if (st) return fail(st, "block %d: %s", i, g_err.c_str());
        st = check_scheme(&fb.grid, &b->sch);
        if (st) return fail(st, "block %d: %s", i, g_err.c_str());
        if (!fb.met || !fb.q || !fb.work) return fail(FP_EINVAL, "block %d: NULL array", i);
        if (!(fb.dt > 0.0)) return fail(FP_EINVAL, "block %d: dt must be positive", i);
    }
    std::vector<fp_block> v(blocks, blocks + nblocks);
    std::vector<fp_link> nolinks;
    st = upload_tables(b, v, nolinks, (hipStream_t)stream);
    if (st) return st;
    b->blocks.swap(v);
    b->links.clear();
    return FP_OK;
}

fp_status fp_batch_rk3_step(fp_batch* b, void* stream) {
    fp_status st = check_batch(b);
    if (st) return st;
    hipError_t e = run_batch_step(b, batch_mask(b), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fp_batch_rk3_step launch");
    return FP_OK;
}

fp_status fp_batch_solve(fp_batch* b, int64_t nsteps, void* stream) {
    fp_status st = check_batch(b);
    if (st) return st;
    if (nsteps < 0) return fail(FP_EINVAL, "nsteps must be >= 0");
    const int mask = batch_mask(b);
    if (nsteps == 0 || mask == 0) return FP_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (!b->graph[mask]) {
        e = hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = run_batch_step(b, mask, b->cs, false);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(b->cs, &graph);
        if (le != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return hip_fail(le, "fp_batch_solve capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        b->graph[mask] = exec;
    }
    run_batch_ghosts(b, mask, s);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp_batch_solve ghost copy");
    for (int64_t i = 0; i < nsteps; ++i) {
        e = hipGraphLaunch(b->graph[mask], s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    return FP_OK;
}

fp_status fp_batch_autotune(fp_batch* b, int32_t* segment, void* stream) {
    fp_status st = check_batch(b);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const int mask = batch_mask(b);
    if (mask == 0) {
        if (segment) *segment = b->seg[1];
        return FP_OK;
    }
    const TuneKey key = tune_key(b);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            b->seg[1] = it->second.first;
            b->seg[2] = it->second.second;
            b->tuned_from_cache = true;
            st = upload_tables(b, b->blocks, b->links, s);
            if (st) return st;
            if (segment) *segment = b->seg[1];
            return FP_OK;
        }
    }
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    // time RK stage 1 (every sweep) of the current blocks for a choice: the
    // fastest of four repetitions after one that warms up (the optimum is
    // flat, so a sum of few repetitions lets run-to-run noise pick)
    auto time_stage = [&](float* out) -> fp_status {
        fp_status r = upload_tables(b, b->blocks, b->links, s);
        if (r) return r;
        float ms = -1.0f;
        for (int rep = 0; rep < 5 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, s);
            for (int p = 0; p < 2 && e == hipSuccess; ++p)
                if (mask & (1 << p)) e = b->fn[p](b->tab[p], b->sk, 0, b->grid[p], -1, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (rep > 0 && (ms < 0.0f || t < ms)) ms = t;
        }
        *out = ms;
        return FP_OK;
    };
    // coordinate search: the eta target with zeta's held, then zeta's (2D
    // blocks have no zeta sweep: their time does not depend on it)
    for (int d = 1; d <= 2 && st == FP_OK && e == hipSuccess; ++d) {
        int best = b->seg[d];
        float best_ms = -1.0f;
        for (int T : kSegTargets) {
            b->seg[d] = T;
            float ms = 0.0f;
            st = time_stage(&ms);
            if (st || e != hipSuccess) break;
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                best = T;
            }
        }
        b->seg[d] = best;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) return st;
    if (e != hipSuccess) return hip_fail(e, "fp_batch_autotune");
    st = upload_tables(b, b->blocks, b->links, s);
    if (st) return st;
    b->tuned_from_cache = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = {b->seg[1], b->seg[2]};
    }
    if (segment) *segment = b->seg[1];
    return FP_OK;
}

fp_status fp_batch_get_tiles(const fp_batch* b, int32_t* seg_eta, int32_t* seg_zeta, int32_t* from_cache) {
    if (!b) return fail(FP_EINVAL, "batch is NULL");
    if (seg_eta) *seg_eta = b->seg[1];
    if (seg_zeta) *seg_zeta = b->seg[2];
    if (from_cache) *from_cache = b->tuned_from_cache ? 1 : 0;
    return FP_OK;
}

fp_status fp_batch_set_links(fp_batch* b, const fp_link* links, int32_t nlinks, void* stream) {
    fp_status st = check_batch(b);
    if (st) return st;
    const int nb = (int)b->blocks.size();
    if (nlinks < 0 || nlinks > b->maxl) return fail(FP_EINVAL, "nlinks must be in [0, %d]", b->maxl);
    if (nlinks > 0 && !links) return fail(FP_EINVAL, "links is NULL");
    std::vector<char> seen((size_t)nb * 6, 0);
    for (int i = 0; i < nlinks; ++i) {
        const fp_link& L = links[i];
        if (L.block < 0 || L.block >= nb || L.nbr < 0 || L.nbr >= nb)
            return fail(FP_EINVAL, "link %d: block index out of range", i);
        const fp_grid& A = b->blocks[L.block].grid;
        const fp_grid& B = b->blocks[L.nbr].grid;
        if (A.ndim != B.ndim) return fail(FP_EINVAL, "link %d: blocks of different dimensionality", i);
        if (L.axis < 0 || L.axis >= A.ndim) return fail(FP_EINVAL, "link %d: axis out of range", i);
        if (L.side != 0 && L.side != 1) return fail(FP_EINVAL, "link %d: side must be 0 or 1", i);
        if (A.ghost != B.ghost) return fail(FP_EINVAL, "link %d: blocks of different ghost width", i);
        if (A.bc[L.axis] != FP_BC_FROZEN || B.bc[L.axis] != FP_BC_FROZEN)
            return fail(FP_EINVAL, "link %d: linked axes must be FP_BC_FROZEN in both blocks", i);
        if (B.n[L.axis] < A.ghost) return fail(FP_EINVAL, "link %d: neighbour thinner than the ghost width", i);
        for (int e = 0; e < A.ndim; ++e)
            if (e != L.axis && A.n[e] != B.n[e])
                return fail(FP_EINVAL, "link %d: blocks differ along axis %d", i, e);
        char& u = seen[(size_t)L.block * 6 + L.axis * 2 + L.side];
        if (u) return fail(FP_EINVAL, "link %d: face linked twice", i);
        u = 1;
    }
    std::vector<fp_link> v(links, links + nlinks);
    hipStream_t s = (hipStream_t)stream;
    st = upload_tables(b, b->blocks, v, s);
    if (st) return st;
    b->links.swap(v);
    // metric ghost layers of the linked faces from the neighbours' interiors,
    // once: both blocks then see the same metrics at every interface node
    for (int p = 0; p < 2; ++p) {
        if (b->nblk[p] == 0) continue;
        hipLaunchKernelGGL(kb_halo, dim3(b->grid[p][BK_GHOST]), dim3(256), 0, s, b->lnk_n[p], b->lnk_start[p],
                           b->lnk[p], b->tab[p].blk, p == 0 ? 2 : 3, 3);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp_batch_set_links launch");
    return FP_OK;
}

fp_status fp_batch_profile_step(fp_batch* b, float* kernel_ms, int32_t* kernel_kind, int32_t max_kernels,
                                int32_t* n_kernels, void* stream) {
    fp_status st = check_batch(b);
    if (st) return st;
    if (!kernel_ms || !kernel_kind || !n_kernels) return fail(FP_EINVAL, "NULL output");
    hipStream_t s = (hipStream_t)stream;
    const int mask = batch_mask(b);
    // the launches of one step, in order: (part, kind, stage)
    int plan[2 * 13][3];
    int n = 0;
    for (int p = 0; p < 2; ++p) {
        if (!(mask & (1 << p))) continue;
        const int ndim = p == 0 ? 2 : 3;
        plan[n][0] = p, plan[n][1] = BK_GHOST, plan[n][2] = -1, ++n;
        for (int k = 0; k < 3; ++k) {
            if (mask & (4 << p)) plan[n][0] = p, plan[n][1] = 4, plan[n][2] = k, ++n;  // interface exchange
            for (int kind = 0; kind < ndim; ++kind) plan[n][0] = p, plan[n][1] = kind, plan[n][2] = k, ++n;
        }
    }
    if (n > max_kernels) return fail(FP_EINVAL, "max_kernels must be >= %d", n);
    hipEvent_t ev[2 * 13 + 1];
    hipError_t e = hipSuccess;
    int made = 0;
    while (made <= n) {
        e = hipEventCreate(&ev[made]);
        if (e != hipSuccess) break;
        ++made;
    }
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        const int p = plan[i][0], kind = plan[i][1], k = plan[i][2];
        if (kind == BK_GHOST)
            hipLaunchKernelGGL(kb_frozen_ghosts, dim3(b->grid[p][BK_GHOST]), dim3(256), 0, s, b->tab[p].nblk,
                               b->tab[p].start, b->tab[p].blk, b->tab[p].cap, p == 0 ? 2 : 3);
        else if (kind == 4)
            hipLaunchKernelGGL(kb_halo, dim3(b->grid[p][BK_GHOST]), dim3(256), 0, s, b->lnk_n[p],
                               b->lnk_start[p], b->lnk[p], b->tab[p].blk, p == 0 ? 2 : 3, k);
        else
            e = b->fn[p](b->tab[p], b->sk, k, b->grid[p], kind, s);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(ev[i + 1], s);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[n]);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        e = hipEventElapsedTime(&kernel_ms[i], ev[i], ev[i + 1]);
        kernel_kind[i] = (plan[i][0] == 0 ? 2 : 3) * 16 + plan[i][1];
    }
    for (int i = 0; i < made; ++i) hipEventDestroy(ev[i]);
    if (e != hipSuccess) return hip_fail(e, "fp_batch_profile_step");
    *n_kernels = n;
    return FP_OK;
}

void fp_batch_destroy(fp_batch* b) {
    if (!b) return;
    hipDeviceSynchronize();
    for (auto& gx : b->graph)
        if (gx) hipGraphExecDestroy(gx);
    if (b->cs) hipStreamDestroy(b->cs);
    if (b->staged) hipEventDestroy(b->staged);
    if (b->hstage) hipHostFree(b->hstage);
    if (b->dmem) hipFree(b->dmem);
    delete b;
}

void fp_release_cache(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_graphs) hipGraphExecDestroy(kv.second);
    g_graphs.clear();
    for (auto& kv : g_bc_graphs) hipGraphExecDestroy(kv.second);
    g_bc_graphs.clear();
}

}  // extern "C"
