// fp_api.hip -- host side of the C ABI declared in include/fp.h: argument
// validation, launch geometry, the RK3 stage sequence and the step-graph
// cache of fp_solve.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "fp.h"
#include "fp_kernels.hpp"
#include "fp_util_kernels.hpp"

namespace fpk {

#define FP_DECL_GET(P, R)                                           \
    stage_fn get_stage_p##P##_r##R(int ndim, int Y);                \
    dir_fn get_dir_p##P##_r##R(int ndim, int Y);                    \
    faceflux_fn get_faceflux_p##P##_r##R(int ndim, int dir, int Y);
FP_DECL_GET(0, 0)
FP_DECL_GET(0, 1)
FP_DECL_GET(1, 0)
FP_DECL_GET(1, 1)
#undef FP_DECL_GET

stage_fn get_stage_fn(int ndim, int recon, int Y, int prec) {
    if (prec == 0) return recon == 0 ? get_stage_p0_r0(ndim, Y) : get_stage_p0_r1(ndim, Y);
    return recon == 0 ? get_stage_p1_r0(ndim, Y) : get_stage_p1_r1(ndim, Y);
}

dir_fn get_dir_fn(int ndim, int recon, int Y, int prec) {
    if (prec == 0) return recon == 0 ? get_dir_p0_r0(ndim, Y) : get_dir_p0_r1(ndim, Y);
    return recon == 0 ? get_dir_p1_r0(ndim, Y) : get_dir_p1_r1(ndim, Y);
}

faceflux_fn get_faceflux_fn(int ndim, int dir, int recon, int Y, int prec) {
    if (prec == 0)
        return recon == 0 ? get_faceflux_p0_r0(ndim, dir, Y) : get_faceflux_p0_r1(ndim, dir, Y);
    return recon == 0 ? get_faceflux_p1_r0(ndim, dir, Y) : get_faceflux_p1_r1(ndim, dir, Y);
}

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
    if (s->recon != FP_WENO5JS && s->recon != FP_LINUP5) return fail(FP_EINVAL, "unknown recon %d", s->recon);
    const int Y = s->metric_order;
    if (Y != 2 && Y != 4 && Y != 6 && Y != 8)
        return fail(FP_EUNSUPPORTED, "metric_order must be 2, 4, 6 or 8 (got %d)", Y);
    if (g->ghost < Y / 2) return fail(FP_EINVAL, "metric_order %d needs ghost >= %d", Y, Y / 2);
    if (s->reformulated != 0 && s->reformulated != 1) return fail(FP_EINVAL, "reformulated must be 0 or 1");
    if (s->precision != FP_FP64 && s->precision != FP_MIXED32)
        return fail(FP_EINVAL, "unknown precision %d", s->precision);
    if (!(s->gamma > 1.0)) return fail(FP_EINVAL, "gamma must exceed 1");
    if (!(s->weno_eps > 0.0)) return fail(FP_EINVAL, "weno_eps must be positive");
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

SchemeK make_sk(const fp_scheme* s) {
    SchemeK k;
    k.gamma = s->gamma;
    k.eps = s->weno_eps;
    k.reform = s->reformulated;
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

EpiK epi(int mode, double* R) {
    EpiK e;
    std::memset(&e, 0, sizeof e);
    e.mode = mode;
    e.R = R;
    return e;
}

// one residual evaluation; the last sweep applies `last`
hipError_t run_residual(const Ctx& c, const double* met, const double* qs, double* R,
                        const EpiK& last, hipStream_t s) {
    SweepArgs a;
    a.G = c.G;
    a.sk = c.sk;
    a.met = met;
    a.qs = qs;
    a.ep_first = epi(EPI_FIRST, R);
    a.ep_mid = epi(EPI_MID, R);
    a.ep_last = last;
    plan_segments(c.G, c.grid.ndim, a);
    return c.stage(a, s);
}

// one TVD RK3 step: q -> A -> B -> q with residual accumulator R; the
// frozen ghost layers of q are copied into A and B first
hipError_t run_rk3(const Ctx& c, const double* met, double* q, double* work, double dt, hipStream_t s) {
    double* A = work;
    double* B = work + c.state_elems;
    double* R = work + 2 * c.state_elems;
    bool frozen = false;
    for (int d = 0; d < c.grid.ndim; ++d) frozen = frozen || c.grid.bc[d] == FP_BC_FROZEN;
    if (frozen) {
        hipLaunchKernelGGL(k_frozen_ghosts, dim3((unsigned)((c.G.vol + 255) / 256)), dim3(256), 0, s,
                           c.G, c.grid.ndim, c.grid.ndim + 2, (const double*)q, A, B);
    }
    const double* metV = met + (size_t)(c.grid.ndim == 3 ? 9 : 4) * c.G.vol;
    const double* in[3] = {q, A, B};
    double* out[3] = {A, B, q};
    const double ca[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    const double cb[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    for (int k = 0; k < 3; ++k) {
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
        a.G = c.G;
        a.sk = c.sk;
        a.met = met;
        a.qs = in[k];
        a.ep_first = epi(EPI_FIRST, R);
        a.ep_mid = epi(EPI_MID, R);
        a.ep_last = e;
        plan_segments(c.G, c.grid.ndim, a);
        hipError_t err = c.stage(a, s);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
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
std::map<int, hipStream_t> g_capture_streams;

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
    return 3 * fp_state_bytes(g);
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
    if (dir < 0 || dir >= g->ndim) return fail(FP_EINVAL, "dir must be in [0, ndim)");
    if (!met || !q || !flux) return fail(FP_EINVAL, "NULL array");
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
    if (!met || !q || !dqdt) return fail(FP_EINVAL, "NULL array");
    if ((const double*)dqdt == q) return fail(FP_EINVAL, "dqdt must not alias q");
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
    if (dir < 0 || dir >= g->ndim) return fail(FP_EINVAL, "dir must be in [0, ndim)");
    if (accumulate != 0 && accumulate != 1) return fail(FP_EINVAL, "accumulate must be 0 or 1");
    if (!met || !q || !acc) return fail(FP_EINVAL, "NULL array");
    if ((const double*)acc == q) return fail(FP_EINVAL, "acc must not alias q");
    dir_fn f = get_dir_fn(g->ndim, sch->recon, sch->metric_order, sch->precision);
    if (!f) return fail(FP_EUNSUPPORTED, "no sweep kernel for this scheme");
    SweepArgs a;
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
    if (!met || !q || !work) return fail(FP_EINVAL, "NULL array");
    if (!(dt > 0.0)) return fail(FP_EINVAL, "dt must be positive");
    hipError_t e = run_rk3(c, met, q, work, dt, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fp_rk3_step launch");
    return FP_OK;
}

fp_status fp_solve(const fp_grid* g, const fp_scheme* sch, const double* met, double* q, double* work,
                   double dt, int64_t nsteps, void* stream) {
    Ctx c;
    fp_status st = make_ctx(g, sch, c);
    if (st) return st;
    if (!met || !q || !work) return fail(FP_EINVAL, "NULL array");
    if (!(dt > 0.0)) return fail(FP_EINVAL, "dt must be positive");
    if (nsteps < 0) return fail(FP_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return FP_OK;
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
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) {
            exec = it->second;
        } else {
            hipStream_t cs;
            auto sit = g_capture_streams.find(dev);
            if (sit == g_capture_streams.end()) {
                e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
                if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
                g_capture_streams[dev] = cs;
            } else {
                cs = sit->second;
            }
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            hipError_t le = run_rk3(c, met, q, work, dt, cs);
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
    for (int64_t i = 0; i < nsteps; ++i) {
        e = hipGraphLaunch(exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
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

void fp_release_cache(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_graphs) hipGraphExecDestroy(kv.second);
    g_graphs.clear();
}

}  // extern "C"
