// hydro_api.hip -- host runtime behind include/hydro.h: patch descriptors,
// workspace carving, stream-ordered launches, the device error latch and
// per-kernel event timing.
#include "hydro.h"
#include "hy_internal.h"
#include "hy_diag.h"
#include "hy_mlp.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

hy_status fail(hy_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

hy_status hip_fail(hipError_t e, const char *where)
{
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return HY_EDEVICE;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr int kTimingPool = 4096;

}  // namespace

struct hy_patch {
    hy_patch_desc d;
    int nv = 0;
    int64_t ncell = 0, vstride = 0;
    char *ws = nullptr;
    hy::DevCtl *ctl = nullptr;
    double *partials = nullptr;
    void *A = nullptr;  // U^n (and U^{n+1}, written in place by stage 2)
    void *B = nullptr;  // U^(1)
    float *slopes = nullptr;
    hy::MlpDevice *mlp = nullptr;
    hy::MlpImage *mlpimg = nullptr;
    bool mlp_set = false;
    hipStream_t stream = nullptr;
    int parity = 0;
    const double *dt_dev = nullptr;  // the step of DT_PTR stages (set by the multilevel recursion)
    // a refined level: the arrays hold `inner` interior cells plus 2 exterior
    // cells on each side of every active dimension; the stages update the
    // interior only (LIM_THETA_PADDED)
    bool padded = false;
    int64_t inner[3] = {1, 1, 1};
    hy::LaunchCfg cfg{64, 8, 32};
    // the HLLC -> HLL switch's own shape: its stage kernels hold more state
    // per thread, which a 32x8 tile at three waves per SIMD affords without
    // spilling (3D FP32)
    hy::LaunchCfg cfg_sw{64, 8, 32};
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev[2];
    int nrec[2] = {0, 0};
    double ms[2] = {0.0, 0.0};
    int64_t launches[2] = {0, 0};
    // hy_advance_graph: the captured steps, one graph per starting parity
    struct GraphKey {
        int nsteps = -1, solver = -1;
        double cfl = 0.0, t_end = 0.0;
        hy::LaunchCfg cfg{0, 0, 0};
    };
    hipStream_t capture = nullptr;
    bool capturing = false;  // no timing events while capturing
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    GraphKey gkey[2];
};

namespace {
// the launch shape a solver's stage kernels take
hy::LaunchCfg &cfg_of(hy_patch *p, int solver)
{
    return solver == HY_HLLC_SWITCH ? p->cfg_sw : p->cfg;
}
}  // namespace

namespace {

int64_t ncells(const hy_patch_desc &d) { return d.n[0] * d.n[1] * d.n[2]; }

hy_status check_desc(const hy_patch_desc *d)
{
    if (!d) return fail(HY_EINVAL, "null descriptor");
    if (d->ndim < 1 || d->ndim > 3) return fail(HY_EINVAL, "ndim must be 1, 2 or 3");
    if (!(d->gamma > 1.0) || !std::isfinite(d->gamma)) return fail(HY_EINVAL, "gamma must be > 1");
    if (d->precision != 32 && d->precision != 64) return fail(HY_EINVAL, "precision must be 32 or 64");
    if (d->limiter != HY_LIM_THETA && d->limiter != HY_LIM_LEARNED) return fail(HY_EINVAL, "unknown limiter");
    if (d->limiter == HY_LIM_THETA && !(d->theta >= 1.0 && d->theta <= 2.0))
        return fail(HY_EINVAL, "theta must lie in [1, 2]");
    if (d->limiter == HY_LIM_LEARNED && d->precision != 32)
        return fail(HY_EUNSUPPORTED, "the learned limiter is built for FP32 only");
    for (int q = 0; q < 3; ++q) {
        if (q < d->ndim) {
            if (d->n[q] < 2) return fail(HY_EINVAL, "active dimensions need n >= 2");
            if (!(d->hi[q] > d->lo[q])) return fail(HY_EINVAL, "hi must exceed lo");
            for (int s = 0; s < 2; ++s)
                if (d->bc[q][s] < 0 || d->bc[q][s] > 2) return fail(HY_EINVAL, "unknown boundary kind");
            if ((d->bc[q][0] == HY_BC_PERIODIC) != (d->bc[q][1] == HY_BC_PERIODIC))
                return fail(HY_EINVAL, "periodic boundaries must be paired");
        } else if (d->n[q] != 1) {
            return fail(HY_EINVAL, "unused dimensions must have n = 1");
        }
        if (!std::isfinite(d->accel[q])) return fail(HY_EINVAL, "accel must be finite");
    }
    if (d->n[0] > (int64_t)1 << 20 || d->n[1] > 65535 || d->n[2] > 65535)
        return fail(HY_EINVAL, "dimension too large (n_x <= 2^20, n_y and n_z <= 65535)");
    const int64_t N = ncells(*d);
    // kernels address cells with 32-bit offsets within one variable's array
    const int64_t es = d->precision == 64 ? 8 : 4;
    if (N * es > ((int64_t)1 << 32) - 256)
        return fail(HY_EINVAL, "patch too large: one variable's array must stay below 4 GiB");
    return HY_OK;
}

struct Layout {
    size_t ctl, partials, A, B, slopes, mlp, mlpimg, total;
    int64_t vstride;
};

Layout layout(const hy_patch_desc &d)
{
    Layout L{};
    const size_t es = d.precision == 64 ? 8 : 4;
    const int nv = d.ndim + 2;
    L.vstride = (int64_t)align_up((size_t)ncells(d), 64);
    size_t o = 0;
    L.ctl = o;
    o = align_up(o + sizeof(hy::DevCtl), 256);
    L.partials = o;
    o = align_up(o + sizeof(double) * 5 * hy::TOTALS_BLOCKS, 256);
    L.mlp = o;
    o = align_up(o + sizeof(hy::MlpDevice), 256);
    L.mlpimg = o;
    o = align_up(o + sizeof(hy::MlpImage), 256);
    L.A = o;
    o = align_up(o + es * nv * (size_t)L.vstride, 256);
    L.B = o;
    o = align_up(o + es * nv * (size_t)L.vstride, 256);
    L.slopes = o;
    if (d.limiter == HY_LIM_LEARNED) o = align_up(o + sizeof(float) * d.ndim * nv * (size_t)L.vstride, 256);
    L.total = o + 256;  // slack for aligning the caller's base pointer
    return L;
}

int stage_limiter(const hy_patch *p) { return p->padded ? hy::LIM_THETA_PADDED : p->d.limiter; }

template <typename T>
hy::StageArgs<T> stage_args(hy_patch *p, int stage, int dt_mode, double dt, double cfl, double t_end)
{
    hy::StageArgs<T> a{};
    const hy_patch_desc &d = p->d;
    T *A = (T *)p->A, *B = (T *)p->B;
    a.uin = stage == 1 ? A : B;
    a.uout = stage == 1 ? B : A;
    a.u0 = A;
    a.slopes = p->slopes;
    for (int q = 0; q < 3; ++q) {
        a.n[q] = p->padded ? p->inner[q] : d.n[q];
        a.voff[q] = p->padded && q < d.ndim ? 2 : 0;  // the interior of a padded level
        a.vm[q] = (int)d.n[q];
        a.idx[q] = q < d.ndim ? (T)((double)d.n[q] / (d.hi[q] - d.lo[q])) : T(0);
        a.accel[q] = q < d.ndim ? (T)d.accel[q] : T(0);
        a.bc[q][0] = d.bc[q][0];
        a.bc[q][1] = d.bc[q][1];
    }
    a.vstride = p->vstride;
    a.gamma = (T)d.gamma;
    a.gm1 = (T)(d.gamma - 1.0);
    a.inv_gm1 = (T)(1.0 / (d.gamma - 1.0));
    a.theta = (T)d.theta;
    a.zchunk = p->cfg.zchunk;
    a.ctl = p->ctl;
    a.parity = p->parity;
    a.dt_mode = dt_mode;
    a.dt_host = dt;
    a.cfl = cfl;
    a.t_end = t_end;
    a.dt_dev = p->dt_dev;
    return a;
}

template <typename T>
hipError_t run_stage(hy_patch *p, int solver, int stage, int dt_mode, double dt, double cfl, double t_end)
{
    hipError_t e;
    if (p->d.limiter == HY_LIM_LEARNED) {
        const T *uin = (const T *)(stage == 1 ? p->A : p->B);
        e = hy::launch_learned_slopes((const float *)uin, p->slopes, p->d.n, p->vstride, p->vstride, p->d.ndim,
                                      (float)(p->d.gamma - 1.0), p->d.bc, p->mlpimg, p->stream);
        if (e != hipSuccess) return e;
    }
    const int k = stage - 1;
    const bool rec = p->timing && !p->capturing && p->nrec[k] < kTimingPool;
    if (rec) {
        e = hipEventRecord(p->ev[k][2 * p->nrec[k]], p->stream);
        if (e != hipSuccess) return e;
    }
    hy::StageArgs<T> a = stage_args<T>(p, stage, dt_mode, dt, cfl, t_end);
    const hy::LaunchCfg &c = cfg_of(p, solver);
    a.zchunk = c.zchunk;
    e = hy::launch_stage<T>(p->d.ndim, solver, stage, stage_limiter(p), c, a, p->stream);
    if (e != hipSuccess) return e;
    if (rec) {
        e = hipEventRecord(p->ev[k][2 * p->nrec[k] + 1], p->stream);
        if (e != hipSuccess) return e;
        p->nrec[k]++;
    }
    return hipSuccess;
}

hipError_t one_step(hy_patch *p, int solver, int dt_mode, double dt, double cfl, double t_end)
{
    hipError_t e;
    if (p->d.precision == 64) {
        e = run_stage<double>(p, solver, 1, dt_mode, dt, cfl, t_end);
        if (e == hipSuccess) e = run_stage<double>(p, solver, 2, dt_mode, dt, cfl, t_end);
    } else {
        e = run_stage<float>(p, solver, 1, dt_mode, dt, cfl, t_end);
        if (e == hipSuccess) e = run_stage<float>(p, solver, 2, dt_mode, dt, cfl, t_end);
    }
    if (e == hipSuccess) p->parity ^= 1;
    return e;
}

// the spectrum's shape checks: a 2D patch of N x N cells (N a power of two,
// 2 .. 8192) on a square box
hy_status spectrum_check(hy_patch *p, int *n_out)
{
    if (!p) return fail(HY_EINVAL, "null patch");
    const hy_patch_desc &d = p->d;
    if (d.ndim != 2 || p->padded) return fail(HY_EUNSUPPORTED, "the spectrum takes a 2D patch");
    const int64_t n = d.n[0];
    if (d.n[1] != n || n < 2 || n > 8192 || (n & (n - 1)) != 0)
        return fail(HY_EUNSUPPORTED, "the spectrum needs N x N cells, N a power of two from 2 to 8192");
    const double lx = d.hi[0] - d.lo[0], ly = d.hi[1] - d.lo[1];
    if (!(std::fabs(lx - ly) <= 1e-12 * std::fmax(lx, ly))) return fail(HY_EUNSUPPORTED, "the spectrum needs a square box");
    *n_out = (int)n;
    return HY_OK;
}

hy_status read_ctl(hy_patch *p, hy::DevCtl *out)
{
    hipError_t e = hipMemcpyAsync(out, p->ctl, sizeof(hy::DevCtl), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "reading the control block");
    return HY_OK;
}

hy_status compute_rate(hy_patch *p)
{
    const hy_patch_desc &d = p->d;
    double idx[3];
    for (int q = 0; q < 3; ++q) idx[q] = q < d.ndim ? (double)d.n[q] / (d.hi[q] - d.lo[q]) : 0.0;
    hipError_t e;
    if (d.precision == 64)
        e = hy::launch_cfl_rate<double>((const double *)p->A, d.n[0], d.n[1], d.n[2], p->vstride, d.ndim, d.gamma,
                                        d.gamma - 1.0, idx, p->ctl, p->parity, p->stream);
    else
        e = hy::launch_cfl_rate<float>((const float *)p->A, d.n[0], d.n[1], d.n[2], p->vstride, d.ndim,
                                       (float)d.gamma, (float)(d.gamma - 1.0), idx, p->ctl, p->parity, p->stream);
    if (e != hipSuccess) return hip_fail(e, "cfl rate launch");
    return HY_OK;
}

// Plane tiles the stage kernels are instantiated for (BX x BY threads).
bool tile_supported(const hy_patch_desc &d, int bx, int by)
{
    if (d.ndim == 1) return bx == 64 && by == 1;
    return (bx == 64 && (by == 8 || by == 4)) || (bx == 32 && (by == 8 || (by == 16 && d.precision == 32)));
}

void pick_config(hy_patch *p)
{
    // plane tile and z chunk: at least ~512 workgroups (two per CU) and at
    // most 64 planes per workgroup (measured best at 256^3: 64x8 tile, 64 planes)
    const hy_patch_desc &d = p->d;
    const int64_t *n = p->padded ? p->inner : d.n;  // the extents the stages cover
    p->cfg.bx = 64;
    p->cfg.by = d.ndim == 1 ? 1 : 8;

    if (const char *e = std::getenv("HY_TILE")) {  // "BXxBY", for tuning runs
        int bx = 0, by = 0;
        if (d.ndim > 1 && std::sscanf(e, "%dx%d", &bx, &by) == 2 && tile_supported(d, bx, by)) {
            p->cfg.bx = bx;
            p->cfg.by = by;
        }
    }
    if (d.ndim == 3) {
        const int64_t tiles = ((n[0] + p->cfg.bx - 1) / p->cfg.bx) * ((n[1] + p->cfg.by - 1) / p->cfg.by);
        int64_t chunks = (512 + tiles - 1) / tiles;
        chunks = std::max<int64_t>(chunks, (n[2] + 63) / 64);
        if (chunks > n[2] / 8) chunks = n[2] / 8;
        if (chunks < 1) chunks = 1;
        p->cfg.zchunk = (int)((n[2] + chunks - 1) / chunks);
        if (const char *e = std::getenv("HY_ZCHUNK")) {  // planes per workgroup, for tuning runs
            const int zc = std::atoi(e);
            if (zc >= 1 && zc <= n[2]) p->cfg.zchunk = zc;
        }
    } else {
        p->cfg.zchunk = 1;
    }
    p->cfg_sw = p->cfg;
    if (d.ndim == 3 && d.precision == 32 && !std::getenv("HY_TILE")) {
        // 32x8 tiles, three per CU: at least ~1536 workgroups (two rounds)
        const int64_t tiles = ((n[0] + 31) / 32) * ((n[1] + 7) / 8);
        int64_t chunks = (1536 + tiles - 1) / tiles;
        chunks = std::max<int64_t>(chunks, (n[2] + 63) / 64);
        if (chunks > n[2] / 8) chunks = n[2] / 8;
        if (chunks < 1) chunks = 1;
        p->cfg_sw = {32, 8, (int)((n[2] + chunks - 1) / chunks)};
        if (const char *e = std::getenv("HY_ZCHUNK")) {
            const int zc = std::atoi(e);
            if (zc >= 1 && zc <= n[2]) p->cfg_sw.zchunk = zc;
        }
    }
}


}  // namespace

namespace {

bool same_key(const hy_patch::GraphKey &k, int nsteps, int solver, double cfl, double t_end, const hy::LaunchCfg &cfg)
{
    return k.nsteps == nsteps && k.solver == solver && k.cfl == cfl && k.t_end == t_end && k.cfg.bx == cfg.bx &&
           k.cfg.by == cfg.by && k.cfg.zchunk == cfg.zchunk;
}

// Folds the timing events of the launches recorded so far into the totals
// (synchronising).
hipError_t fold_times(hy_patch *p)
{
    if (p->nrec[0] == 0 && p->nrec[1] == 0) return hipSuccess;
    hipError_t e = hipStreamSynchronize(p->stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        for (int i = 0; i < p->nrec[k] && e == hipSuccess; ++i) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, p->ev[k][2 * i], p->ev[k][2 * i + 1]);
            p->ms[k] += t;
        }
        p->launches[k] += p->nrec[k];
        p->nrec[k] = 0;
    }
    return e;
}

// Captures nsteps device-dt steps from the current parity into
// p->gexec[parity] (kernel launches only: no memset, event or host wait).
// Nothing runs.
hy_status capture_steps(hy_patch *p, int nsteps, int solver, double cfl, double t_end)
{
    const int par = p->parity;
    if (p->gexec[par]) (void)hipGraphExecDestroy(p->gexec[par]);
    p->gexec[par] = nullptr;
    p->gkey[par] = hy_patch::GraphKey{};
    hipError_t e = hipSuccess;
    if (!p->capture) e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    hipStream_t caller = p->stream;
    e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    p->stream = p->capture;
    p->capturing = true;
    hipError_t el = hipSuccess;
    for (int i = 0; i < nsteps && el == hipSuccess; ++i) el = one_step(p, solver, hy::DT_DEVICE, 0.0, cfl, t_end);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->capture, &g);
    p->capturing = false;
    p->stream = caller;
    p->parity = par;  // captured, not run
    if (el != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(el != hipSuccess ? el : e, "step capture");
    }
    e = hipGraphInstantiate(&p->gexec[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        p->gexec[par] = nullptr;
        return hip_fail(e, "graph instantiate");
    }
    hy_patch::GraphKey &k = p->gkey[par];
    k.nsteps = nsteps;
    k.solver = solver;
    k.cfl = cfl;
    k.t_end = t_end;
    k.cfg = cfg_of(p, solver);
    return HY_OK;
}

hy_status check_advance(hy_patch *p, int nsteps, double cfl, double t_end, int solver)
{
    if (!p) return fail(HY_EINVAL, "null patch");
    if (nsteps < 0) return fail(HY_EINVAL, "nsteps must be >= 0");
    if (!(cfl > 0.0) || !std::isfinite(cfl) || std::isnan(t_end)) return fail(HY_EINVAL, "bad cfl or t_end");
    if (solver != HY_HLL && solver != HY_HLLC && solver != HY_HLLC_SWITCH) return fail(HY_EINVAL, "unknown solver");
    if (p->d.limiter == HY_LIM_LEARNED && !p->mlp_set) return fail(HY_EINVAL, "learned limiter without weights");
    return HY_OK;
}

}  // namespace

extern "C" {

const char *hy_last_error(void) { return g_err.c_str(); }

hy_status hy_patch_workspace_bytes(const hy_patch_desc *desc, size_t *bytes)
{
    hy_status st = check_desc(desc);
    if (st != HY_OK) return st;
    if (!bytes) return fail(HY_EINVAL, "null output");
    *bytes = layout(*desc).total;
    return HY_OK;
}

hy_status hy_init_patch(const hy_patch_desc *desc, void *dev_workspace, size_t bytes, void *hip_stream,
                        hy_patch **out)
{
    hy_status st = check_desc(desc);
    if (st != HY_OK) return st;
    if (!out || !dev_workspace) return fail(HY_EINVAL, "null workspace or output handle");
    Layout L = layout(*desc);
    if (bytes < L.total) return fail(HY_ENOMEM, "workspace too small");
    hy_patch *p = new (std::nothrow) hy_patch();
    if (!p) return fail(HY_ENOMEM, "host allocation failed");
    p->d = *desc;
    p->nv = desc->ndim + 2;
    p->ncell = ncells(*desc);
    p->vstride = L.vstride;
    char *base = (char *)(((uintptr_t)dev_workspace + 255) & ~(uintptr_t)255);
    p->ws = base;
    p->ctl = (hy::DevCtl *)(base + L.ctl);
    p->partials = (double *)(base + L.partials);
    p->mlp = (hy::MlpDevice *)(base + L.mlp);
    p->mlpimg = (hy::MlpImage *)(base + L.mlpimg);
    p->A = base + L.A;
    p->B = base + L.B;
    p->slopes = desc->limiter == HY_LIM_LEARNED ? (float *)(base + L.slopes) : nullptr;
    p->stream = (hipStream_t)hip_stream;
    pick_config(p);
    hipError_t e = hy::launch_ctl_init(p->ctl, p->stream);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "control block init");
    }
    *out = p;
    return HY_OK;
}

hy_status hy_set_state(hy_patch *p, int kind, const double *host)
{
    if (!p || !host) return fail(HY_EINVAL, "null argument");
    if (kind != HY_PRIMITIVE && kind != HY_CONSERVED) return fail(HY_EINVAL, "unknown state kind");
    const int64_t N = p->ncell;
    const size_t es = p->d.precision == 64 ? 8 : 4;
    std::vector<char> stage(es * (size_t)p->nv * (size_t)p->vstride, 0);
    for (int v = 0; v < p->nv; ++v)
        for (int64_t c = 0; c < N; ++c) {
            const double x = host[(int64_t)v * N + c];
            if (es == 8) ((double *)stage.data())[v * p->vstride + c] = x;
            else ((float *)stage.data())[v * p->vstride + c] = (float)x;
        }
    hipError_t e = hipMemcpyAsync(p->A, stage.data(), stage.size(), hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "state upload");
    if (kind == HY_PRIMITIVE) {
        const double gm1 = p->d.gamma - 1.0;
        if (es == 8) e = hy::launch_prim_to_cons<double>((double *)p->A, N, p->vstride, p->d.ndim, gm1, 1.0 / gm1, p->stream);
        else e = hy::launch_prim_to_cons<float>((float *)p->A, N, p->vstride, p->d.ndim, (float)gm1, (float)(1.0 / gm1), p->stream);
        if (e != hipSuccess) return hip_fail(e, "prim_to_cons launch");
    }
    p->parity = 0;
    e = hy::launch_ctl_init(p->ctl, p->stream);
    if (e != hipSuccess) return hip_fail(e, "control block init");
    hy_status st = compute_rate(p);
    if (st != HY_OK) return st;
    hy::DevCtl c;
    st = read_ctl(p, &c);
    if (st != HY_OK) return st;
    if (c.err) return fail(HY_ESTATE, "state holds rho <= 0, p <= 0 or a non-finite value");
    return HY_OK;
}

hy_status hy_get_state(hy_patch *p, int kind, double *out)
{
    if (!p || !out) return fail(HY_EINVAL, "null argument");
    if (kind != HY_PRIMITIVE && kind != HY_CONSERVED) return fail(HY_EINVAL, "unknown state kind");
    const int64_t N = p->ncell;
    const size_t es = p->d.precision == 64 ? 8 : 4;
    const void *src = p->A;
    hipError_t e = hipSuccess;
    if (kind == HY_PRIMITIVE) {
        const double gm1 = p->d.gamma - 1.0;
        if (es == 8) e = hy::launch_cons_to_prim<double>((const double *)p->A, (double *)p->B, N, p->vstride, p->d.ndim, gm1, p->stream);
        else e = hy::launch_cons_to_prim<float>((const float *)p->A, (float *)p->B, N, p->vstride, p->d.ndim, (float)gm1, p->stream);
        if (e != hipSuccess) return hip_fail(e, "cons_to_prim launch");
        src = p->B;
    }
    std::vector<char> stage(es * (size_t)p->nv * (size_t)p->vstride);
    e = hipMemcpyAsync(stage.data(), src, stage.size(), hipMemcpyDeviceToHost, p->stream);
    if (e != hipSuccess) return hip_fail(e, "state download");
    hy::DevCtl c;
    hy_status st = read_ctl(p, &c);
    if (st != HY_OK) return st;
    for (int v = 0; v < p->nv; ++v)
        for (int64_t i = 0; i < N; ++i)
            out[(int64_t)v * N + i] = es == 8 ? ((const double *)stage.data())[v * p->vstride + i]
                                              : (double)((const float *)stage.data())[v * p->vstride + i];
    if (c.err) return fail(HY_ESTATE, "a kernel met rho <= 0, p <= 0 or a non-finite value");
    return HY_OK;
}

hy_status hy_step(hy_patch *p, double dt, int solver)
{
    if (!p) return fail(HY_EINVAL, "null patch");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HY_EINVAL, "dt must be finite and > 0");
    if (solver != HY_HLL && solver != HY_HLLC && solver != HY_HLLC_SWITCH) return fail(HY_EINVAL, "unknown solver");
    if (p->d.limiter == HY_LIM_LEARNED && !p->mlp_set) return fail(HY_EINVAL, "learned limiter without weights");
    hipError_t e = one_step(p, solver, hy::DT_HOST, dt, 0.0, 0.0);
    if (e != hipSuccess) return hip_fail(e, "stage launch");
    return HY_OK;
}

hy_status hy_advance(hy_patch *p, int nsteps, double cfl, double t_end, int solver)
{
    hy_status st = check_advance(p, nsteps, cfl, t_end, solver);
    if (st != HY_OK) return st;
    for (int i = 0; i < nsteps; ++i) {
        hipError_t e = one_step(p, solver, hy::DT_DEVICE, 0.0, cfl, t_end);
        if (e != hipSuccess) return hip_fail(e, "stage launch");
    }
    return HY_OK;
}

hy_status hy_advance_graph_prepare(hy_patch *p, int nsteps, double cfl, double t_end, int solver)
{
    hy_status st = check_advance(p, nsteps, cfl, t_end, solver);
    if (st != HY_OK) return st;
    if (p->padded) return fail(HY_EUNSUPPORTED, "refined levels step through the multilevel calls");
    if (p->gexec[p->parity] && same_key(p->gkey[p->parity], nsteps, solver, cfl, t_end, cfg_of(p, solver))) return HY_OK;
    return capture_steps(p, nsteps, solver, cfl, t_end);
}

hy_status hy_advance_graph(hy_patch *p, int nsteps, double cfl, double t_end, int solver)
{
    hy_status st = hy_advance_graph_prepare(p, nsteps, cfl, t_end, solver);
    if (st != HY_OK) return st;
    hipError_t e = hipGraphLaunch(p->gexec[p->parity], p->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    if (nsteps & 1) p->parity ^= 1;
    return HY_OK;
}

hy_status hy_cfl_dt(hy_patch *p, double cfl, double *dt_out)
{
    if (!p || !dt_out) return fail(HY_EINVAL, "null argument");
    if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(HY_EINVAL, "cfl must be finite and > 0");
    hy::DevCtl c;
    hy_status st = read_ctl(p, &c);
    if (st != HY_OK) return st;
    unsigned long long rb = 0ull;
    for (int k = 0; k < hy::RATE_SLOTS; ++k) rb = std::max(rb, c.rate[p->parity][k]);
    const double rate = __builtin_bit_cast(double, rb);
    *dt_out = cfl / rate;
    if (c.err || !(rate > 0.0) || !std::isfinite(rate))
        return fail(HY_ESTATE, "a kernel met rho <= 0, p <= 0 or a non-finite value");
    return HY_OK;
}

hy_status hy_get_time(hy_patch *p, double *t_out)
{
    if (!p || !t_out) return fail(HY_EINVAL, "null argument");
    hy::DevCtl c;
    hy_status st = read_ctl(p, &c);
    if (st != HY_OK) return st;
    *t_out = c.time[p->parity];
    return c.err ? fail(HY_ESTATE, "a kernel met rho <= 0, p <= 0 or a non-finite value") : HY_OK;
}

hy_status hy_conserved_totals(hy_patch *p, double out[5])
{
    if (!p || !out) return fail(HY_EINVAL, "null argument");
    double dv = 1.0;
    for (int q = 0; q < p->d.ndim; ++q) dv *= (p->d.hi[q] - p->d.lo[q]) / (double)p->d.n[q];
    hipError_t e;
    if (p->d.precision == 64)
        e = hy::launch_totals<double>((const double *)p->A, p->ncell, p->vstride, p->d.ndim, dv, p->partials,
                                      hy::TOTALS_BLOCKS, p->ctl, p->stream);
    else
        e = hy::launch_totals<float>((const float *)p->A, p->ncell, p->vstride, p->d.ndim, dv, p->partials,
                                     hy::TOTALS_BLOCKS, p->ctl, p->stream);
    if (e != hipSuccess) return hip_fail(e, "totals launch");
    hy::DevCtl c;
    hy_status st = read_ctl(p, &c);
    if (st != HY_OK) return st;
    for (int k = 0; k < 5; ++k) out[k] = c.totals[k];
    return c.err ? fail(HY_ESTATE, "a kernel met rho <= 0, p <= 0 or a non-finite value") : HY_OK;
}

hy_status hy_kinetic_energy(hy_patch *p, double out[3])
{
    if (!p || !out) return fail(HY_EINVAL, "null argument");
    double dv = 1.0;
    for (int q = 0; q < p->d.ndim; ++q) dv *= (p->d.hi[q] - p->d.lo[q]) / (double)p->d.n[q];
    hipError_t e;
    if (p->d.precision == 64)
        e = hy::launch_kinetic<double>((const double *)p->A, p->ncell, p->vstride, p->d.ndim, dv, p->partials,
                                       hy::TOTALS_BLOCKS, p->ctl, p->stream);
    else
        e = hy::launch_kinetic<float>((const float *)p->A, p->ncell, p->vstride, p->d.ndim, dv, p->partials,
                                      hy::TOTALS_BLOCKS, p->ctl, p->stream);
    if (e != hipSuccess) return hip_fail(e, "kinetic energy launch");
    hy::DevCtl c;
    hy_status st = read_ctl(p, &c);
    if (st != HY_OK) return st;
    for (int q = 0; q < 3; ++q) out[q] = c.totals[5 + q];
    return c.err ? fail(HY_ESTATE, "a kernel met rho <= 0, p <= 0 or a non-finite value") : HY_OK;
}

hy_status hy_spectrum_workspace_bytes(hy_patch *p, size_t *bytes)
{
    if (!bytes) return fail(HY_EINVAL, "null output");
    int n = 0;
    hy_status st = spectrum_check(p, &n);
    if (st != HY_OK) return st;
    *bytes = hy::spectrum_workspace_bytes(n);
    return HY_OK;
}

hy_status hy_kinetic_spectrum(hy_patch *p, void *dev_workspace, size_t bytes, double *e, int cap, int *nshell)
{
    int n = 0;
    hy_status st = spectrum_check(p, &n);
    if (st != HY_OK) return st;
    if (!dev_workspace || !e || !nshell) return fail(HY_EINVAL, "null argument");
    const int ns = hy::spectrum_shells(n);
    *nshell = ns;
    if (cap < ns) return fail(HY_EINVAL, "output shorter than the shell count");
    if (bytes < hy::spectrum_workspace_bytes(n)) return fail(HY_ENOMEM, "workspace too small");
    const double box = p->d.hi[0] - p->d.lo[0];
    double *e_dev = nullptr;
    hipError_t err = p->d.precision == 64
                         ? hy::launch_spectrum<double>((const double *)p->A, p->vstride, n, box, dev_workspace, &e_dev,
                                                       p->ctl, p->stream)
                         : hy::launch_spectrum<float>((const float *)p->A, p->vstride, n, box, dev_workspace, &e_dev,
                                                      p->ctl, p->stream);
    if (err == hipSuccess) err = hipMemcpyAsync(e, e_dev, (size_t)ns * sizeof(double), hipMemcpyDeviceToHost, p->stream);
    if (err != hipSuccess) return hip_fail(err, "spectrum launch");
    hy::DevCtl c;
    st = read_ctl(p, &c);
    if (st != HY_OK) return st;
    return c.err ? fail(HY_ESTATE, "a kernel met rho <= 0, p <= 0 or a non-finite value") : HY_OK;
}

hy_status hy_set_mlp(hy_patch *p, const float *w, size_t n)
{
    if (!p || !w) return fail(HY_EINVAL, "null argument");
    if (n != (size_t)hy::MLP_NPARAM) return fail(HY_EINVAL, "expected 1249 weights");
    hy::MlpDevice host;
    hy::mlp_pack(w, &host);
    hipError_t e = hipMemcpyAsync(p->mlp, &host, sizeof(host), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hy::launch_mlp_image(p->mlp, p->mlpimg, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "weight upload");
    p->mlp_set = true;
    return HY_OK;
}

hy_status hy_set_timing(hy_patch *p, int on)
{
    if (!p) return fail(HY_EINVAL, "null patch");
    if (on && p->ev[0].empty()) {
        for (int k = 0; k < 2; ++k) {
            p->ev[k].resize(2 * kTimingPool);
            for (auto &ev : p->ev[k]) {
                hipError_t e = hipEventCreate(&ev);
                if (e != hipSuccess) return hip_fail(e, "event create");
            }
        }
    }
    p->timing = on != 0;
    return HY_OK;
}

hy_status hy_kernel_times(hy_patch *p, double ms[2], int64_t launches[2])
{
    if (!p || !ms || !launches) return fail(HY_EINVAL, "null argument");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess) e = fold_times(p);
    if (e != hipSuccess) return hip_fail(e, "event timing");
    for (int k = 0; k < 2; ++k) {
        ms[k] = p->ms[k];
        launches[k] = p->launches[k];
        p->ms[k] = 0.0;
        p->launches[k] = 0;
    }
    return HY_OK;
}

hy_status hy_kernel_config(hy_patch *p, char *buf, size_t len)
{
    if (!p || !buf || len == 0) return fail(HY_EINVAL, "null argument");
    std::snprintf(buf, len, "k_stage<nd=%d,%s,tile=%dx%d> zchunk=%d", p->d.ndim, p->d.precision == 64 ? "f64" : "f32",
                  p->cfg.bx, p->cfg.by, p->cfg.zchunk);
    return HY_OK;
}

hy_status hy_get_launch_cfg(hy_patch *p, hy_launch_cfg *out)
{
    if (!p || !out) return fail(HY_EINVAL, "null argument");
    out->bx = p->cfg.bx;
    out->by = p->cfg.by;
    out->zchunk = p->cfg.zchunk;
    return HY_OK;
}

hy_status hy_set_launch_cfg(hy_patch *p, const hy_launch_cfg *cfg)
{
    if (!p || !cfg) return fail(HY_EINVAL, "null argument");
    if (!tile_supported(p->d, cfg->bx, cfg->by)) return fail(HY_EINVAL, "unsupported plane tile");
    const int64_t zmax = p->d.ndim == 3 ? p->d.n[2] : 1;
    if (cfg->zchunk < 1 || cfg->zchunk > zmax || (p->d.ndim < 3 && cfg->zchunk != 1))
        return fail(HY_EINVAL, "z chunk out of range");
    p->cfg.bx = cfg->bx;
    p->cfg.by = cfg->by;
    p->cfg.zchunk = cfg->zchunk;
    p->cfg_sw = p->cfg;
    return HY_OK;
}

hy_status hy_autotune(hy_patch *p, int solver, int reps, hy_launch_cfg *best, double *best_ms)
{
    if (!p) return fail(HY_EINVAL, "null patch");
    if (solver != HY_HLL && solver != HY_HLLC && solver != HY_HLLC_SWITCH) return fail(HY_EINVAL, "unknown solver");
    if (reps < 1 || reps > 1000) return fail(HY_EINVAL, "reps must be in 1..1000");
    if (p->d.limiter == HY_LIM_LEARNED && !p->mlp_set) return fail(HY_EINVAL, "learned limiter without weights");
    const hy_patch_desc &d = p->d;
    // candidates: every supported tile, and for 3D the z chunks 8..128 that
    // fit plus the default rule's own choice
    std::vector<hy::LaunchCfg> cand;
    const int tiles[4][2] = {{64, 8}, {64, 4}, {32, 8}, {32, 16}};
    hy::LaunchCfg &cur = cfg_of(p, solver);
    const hy::LaunchCfg dflt = cur;
    for (const auto &t : tiles) {
        const int bx = d.ndim == 1 ? 64 : t[0], by = d.ndim == 1 ? 1 : t[1];
        if (!tile_supported(d, bx, by)) continue;
        if (d.ndim == 3) {
            for (int zc : {8, 16, 32, 64, 128})
                if (zc <= d.n[2]) cand.push_back({bx, by, zc});
            if (dflt.zchunk != 8 && dflt.zchunk != 16 && dflt.zchunk != 32 && dflt.zchunk != 64 && dflt.zchunk != 128)
                cand.push_back({bx, by, dflt.zchunk});
        } else {
            cand.push_back({bx, by, 1});
        }
        if (d.ndim == 1) break;
    }
    hipEvent_t ev[2];
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) return hip_fail(e, "event create");
    if (d.limiter == HY_LIM_LEARNED)  // stage 1 reads the slopes of U^n
        e = hy::launch_learned_slopes((const float *)p->A, p->slopes, d.n, p->vstride, p->vstride, d.ndim,
                                      (float)(d.gamma - 1.0), d.bc, p->mlpimg, p->stream);
    // One trial = the two stages of a step with dt = 0, both reading U^n and
    // writing only the scratch state U^(1) (the second stage with U^n as its
    // input and as its U^n term, so it does the second stage's full work);
    // they touch only the control block's slots for the next parity, which
    // the next step's first stage resets.  U^n, the time and the rate of U^n
    // are left as they were.
    auto launch = [&](const hy::LaunchCfg &c) {
        hipError_t r = hipSuccess;
        for (int stage = 1; stage <= 2 && r == hipSuccess; ++stage) {
            if (d.precision == 64) {
                hy::StageArgs<double> a = stage_args<double>(p, stage, hy::DT_HOST, 0.0, 0.0, 0.0);
                a.uin = a.u0 = (const double *)p->A;
                a.uout = (double *)p->B;
                a.zchunk = c.zchunk;
                r = hy::launch_stage<double>(d.ndim, solver, stage, stage_limiter(p), c, a, p->stream);
            } else {
                hy::StageArgs<float> a = stage_args<float>(p, stage, hy::DT_HOST, 0.0, 0.0, 0.0);
                a.uin = a.u0 = (const float *)p->A;
                a.uout = (float *)p->B;
                a.zchunk = c.zchunk;
                r = hy::launch_stage<float>(d.ndim, solver, stage, stage_limiter(p), c, a, p->stream);
            }
        }
        return r;
    };
    // the clocks settle on a few trials of the starting shape first; then two
    // passes over the candidates, each candidate's faster pass counting, and
    // the starting shape is kept unless another is at least 2 % faster
    for (int r = 0; r < 4 * reps && e == hipSuccess; ++r) e = launch(dflt);
    std::vector<double> tms(cand.size(), 1e300);
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        for (size_t k = 0; k < cand.size(); ++k) {
            if (e == hipSuccess) e = launch(cand[k]);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(ev[0], p->stream);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(cand[k]);
            if (e == hipSuccess) e = hipEventRecord(ev[1], p->stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e != hipSuccess) break;
            tms[k] = std::min(tms[k], (double)ms / reps);
        }
    }
    double bms = 1e300, dms = 1e300;
    hy::LaunchCfg bcfg = dflt;
    for (size_t k = 0; k < cand.size(); ++k) {
        const auto &c = cand[k];
        if (c.bx == dflt.bx && c.by == dflt.by && c.zchunk == dflt.zchunk) dms = tms[k];
        if (tms[k] < bms) {
            bms = tms[k];
            bcfg = c;
        }
    }
    if (dms < 1e300 && bms > 0.98 * dms) {
        bcfg = dflt;
        bms = dms;
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    cur = e == hipSuccess ? bcfg : dflt;
    if (e != hipSuccess) return hip_fail(e, "autotune launches");
    if (best) {
        best->bx = bcfg.bx;
        best->by = bcfg.by;
        best->zchunk = bcfg.zchunk;
    }
    if (best_ms) *best_ms = bms;
    return HY_OK;
}

hy_status hy_destroy(hy_patch *p)
{
    if (!p) return HY_OK;
    hipStreamSynchronize(p->stream);
    for (int k = 0; k < 2; ++k) {
        if (p->gexec[k]) hipGraphExecDestroy(p->gexec[k]);
        for (auto &ev : p->ev[k]) hipEventDestroy(ev);
    }
    if (p->capture) hipStreamDestroy(p->capture);
    delete p;
    return HY_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Batched 1D tubes
// ------------------------------------------------------------------------
#include "hy_batch.h"

#include <algorithm>
#include <numeric>

// Per-tube step cap: a bound every workgroup's time loop reaches even if a
// tube's CFL rate blows up (the tube is then flagged as stopped early).
constexpr int kBatchMaxSteps = 400000;

struct hy_batch {
    int count = 0;
    int nmax = 0;
    int64_t ntot = 0;
    std::vector<hy_patch_desc> d;
    std::vector<int64_t> off;
    std::vector<double> cost;  // scheduling estimate n * (n * max signal speed) of each tube
    char *ws = nullptr;
    hy::BatchCtl *ctl = nullptr;
    hy::TubeDesc *tubes = nullptr;
    int *order = nullptr;
    hy::TubeStatus *status = nullptr;
    float *U = nullptr;
    float *W = nullptr;  // scratch for primitive read-back
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    hipGraphExec_t exec = nullptr;
    int nblocks = 0;
    int bt = 1024;  // threads per workgroup of the batched kernel
    int cus = 1;
    bool order_set = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
};

namespace {

struct BatchLayout {
    size_t ctl, tubes, order, status, U, W, total;
    int64_t ntot;
    int nmax;
};

hy_status batch_layout(const hy_patch_desc *descs, int count, BatchLayout *L)
{
    if (!descs || count < 1) return fail(HY_EINVAL, "need at least one tube");
    int64_t ntot = 0;
    int nmax = 0;
    for (int i = 0; i < count; ++i) {
        hy_status st = check_desc(&descs[i]);
        if (st != HY_OK) return st;
        const hy_patch_desc &d = descs[i];
        if (d.ndim != 1 || d.precision != 32 || d.limiter != HY_LIM_THETA)
            return fail(HY_EUNSUPPORTED, "batched tubes are 1D, FP32, generalised-minmod");
        if (d.accel[0] != 0.0) return fail(HY_EUNSUPPORTED, "batched tubes carry no source term");
        if (d.n[0] > hy::BATCH_NMAX) return fail(HY_EINVAL, "tube longer than 6144 cells");
        ntot += d.n[0];
        nmax = std::max(nmax, (int)d.n[0]);
    }
    size_t o = 0;
    L->ctl = o;
    o = align_up(o + sizeof(hy::BatchCtl), 256);
    L->tubes = o;
    o = align_up(o + sizeof(hy::TubeDesc) * count, 256);
    L->order = o;
    o = align_up(o + sizeof(int) * count, 256);
    L->status = o;
    o = align_up(o + sizeof(hy::TubeStatus) * count, 256);
    L->U = o;
    o = align_up(o + sizeof(float) * 3 * (size_t)ntot, 256);
    L->W = o;
    o = align_up(o + sizeof(float) * 3 * (size_t)ntot, 256);
    L->total = o + 256;
    L->ntot = ntot;
    L->nmax = nmax;
    return HY_OK;
}

}  // namespace

extern "C" {

hy_status hy_batch_workspace_bytes(const hy_patch_desc *descs, int count, size_t *bytes)
{
    if (!bytes) return fail(HY_EINVAL, "null output");
    BatchLayout L;
    hy_status st = batch_layout(descs, count, &L);
    if (st != HY_OK) return st;
    *bytes = L.total;
    return HY_OK;
}

hy_status hy_batch_init(const hy_patch_desc *descs, int count, void *dev_workspace, size_t bytes, void *hip_stream,
                        hy_batch **out)
{
    if (!out || !dev_workspace) return fail(HY_EINVAL, "null workspace or output handle");
    BatchLayout L;
    hy_status st = batch_layout(descs, count, &L);
    if (st != HY_OK) return st;
    if (bytes < L.total) return fail(HY_ENOMEM, "workspace too small");
    hy_batch *b = new (std::nothrow) hy_batch();
    if (!b) return fail(HY_ENOMEM, "host allocation failed");
    b->count = count;
    b->nmax = L.nmax;
    b->ntot = L.ntot;
    b->d.assign(descs, descs + count);
    b->off.resize(count);
    b->cost.assign(count, 0.0);
    char *base = (char *)(((uintptr_t)dev_workspace + 255) & ~(uintptr_t)255);
    b->ws = base;
    b->ctl = (hy::BatchCtl *)(base + L.ctl);
    b->tubes = (hy::TubeDesc *)(base + L.tubes);
    b->order = (int *)(base + L.order);
    b->status = (hy::TubeStatus *)(base + L.status);
    b->U = (float *)(base + L.U);
    b->W = (float *)(base + L.W);
    b->stream = (hipStream_t)hip_stream;
    std::vector<hy::TubeDesc> td(count);
    int64_t o = 0;
    for (int i = 0; i < count; ++i) {
        const hy_patch_desc &d = descs[i];
        td[i].n = (int)d.n[0];
        td[i].bclo = d.bc[0][0];
        td[i].bchi = d.bc[0][1];
        td[i].idx = (float)((double)d.n[0] / (d.hi[0] - d.lo[0]));
        td[i].gamma = (float)d.gamma;
        td[i].theta = (float)d.theta;
        td[i].off = o;
        b->off[i] = o;
        o += d.n[0];
    }
    std::vector<int> ord(count);
    std::iota(ord.begin(), ord.end(), 0);
    hy::BatchCtl c{};
    c.max_steps = kBatchMaxSteps;
    // every tube's status starts as "no step taken, no error": the
    // workspace is the caller's memory and may hold anything
    const std::vector<hy::TubeStatus> st0(count, hy::TubeStatus{});
    int dev = 0, cus = 0;
    hipError_t e = hipMemcpyAsync(b->tubes, td.data(), sizeof(hy::TubeDesc) * count, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->order, ord.data(), sizeof(int) * count, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->status, st0.data(), sizeof(hy::TubeStatus) * count, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->ctl, &c, sizeof(c), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hy::prepare_batch(b->nmax);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipEventCreate(&b->ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&b->ev[1]);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch init");
    }
    b->cus = std::max(1, cus);
    b->nblocks = std::min(count, b->cus * hy::batch_blocks_per_cu(b->nmax, b->bt));
    *out = b;
    return HY_OK;
}

hy_status hy_batch_set_state(hy_batch *b, int i, int kind, const double *host)
{
    if (!b || !host) return fail(HY_EINVAL, "null argument");
    if (i < 0 || i >= b->count) return fail(HY_EINVAL, "tube index out of range");
    if (kind != HY_PRIMITIVE && kind != HY_CONSERVED) return fail(HY_EINVAL, "unknown state kind");
    const int64_t n = b->d[i].n[0];
    std::vector<float> st(3 * n);
    for (int64_t k = 0; k < 3 * n; ++k) st[k] = (float)host[k];
    hipError_t e = hipSuccess;
    for (int v = 0; v < 3 && e == hipSuccess; ++v)
        e = hipMemcpyAsync(b->U + v * b->ntot + b->off[i], st.data() + v * n, sizeof(float) * n, hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess && kind == HY_PRIMITIVE) {
        const double gm1 = b->d[i].gamma - 1.0;
        e = hy::launch_prim_to_cons<float>(b->U + b->off[i], n, b->ntot, 1, (float)gm1, (float)(1.0 / gm1), b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "tube upload");
    // scheduling estimate only: tube length times the cells a signal crosses
    // per unit time, n (|v| + c) / L, from the input primitives or conserved
    // variables (the kernel recomputes everything it uses)
    double smax = 0.0;
    const double g = b->d[i].gamma;
    for (int64_t k = 0; k < n; ++k) {
        double rho, v, p;
        if (kind == HY_PRIMITIVE) {
            rho = host[k]; v = host[n + k]; p = host[2 * n + k];
        } else {
            rho = host[k]; v = host[n + k] / rho; p = (g - 1.0) * (host[2 * n + k] - 0.5 * host[n + k] * v);
        }
        const double s = std::fabs(v) + std::sqrt(std::max(g * p / rho, 0.0));
        if (std::isfinite(s)) smax = std::max(smax, s);
    }
    b->cost[i] = (double)n * (double)n * smax / (b->d[i].hi[0] - b->d[i].lo[0]);
    b->order_set = false;
    return HY_OK;
}

// queue order: tubes by descending cost estimate (longest first)
static hy_status batch_order(hy_batch *b)
{
    if (b->order_set) return HY_OK;
    std::vector<int> ord(b->count);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return b->cost[x] > b->cost[y]; });
    hipError_t e = hipMemcpyAsync(b->order, ord.data(), sizeof(int) * b->count, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "queue order upload");
    b->order_set = true;
    return HY_OK;
}

static hy_status batch_capture(hy_batch *b)
{
    hipError_t e = hipSuccess;
    if (!b->capture) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    hipError_t e1 = hy::launch_batch_reset(b->ctl, b->capture);
    hipError_t e2 = hy::launch_batch(b->tubes, b->order, b->U, b->ntot, b->ctl, b->status, b->count, b->nmax,
                                     b->nblocks, b->bt, b->capture);
    e = hipStreamEndCapture(b->capture, &g);
    if (e1 != hipSuccess) e = e1;
    if (e2 != hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    return HY_OK;
}

hy_status hy_batch_run_to(hy_batch *b, double t_end, double cfl, int solver)
{
    if (!b) return fail(HY_EINVAL, "null batch");
    if (!(t_end > 0.0) || !std::isfinite(t_end)) return fail(HY_EINVAL, "t_end must be finite and > 0");
    if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(HY_EINVAL, "cfl must be finite and > 0");
    if (solver != HY_HLL && solver != HY_HLLC && solver != HY_HLLC_SWITCH) return fail(HY_EINVAL, "unknown solver");
    hy_status st0 = batch_order(b);
    if (st0 != HY_OK) return st0;
    hipError_t e = hipSuccess;
    if (!b->exec) {
        hy_status st = batch_capture(b);
        if (st != HY_OK) return st;
    }
    hy::BatchCtl c{};
    c.solver = solver == HY_HLLC_SWITCH ? HY_HLLC : solver;  // no transverse faces in 1D
    c.max_steps = kBatchMaxSteps;
    c.t_end = t_end;
    c.cfl = cfl;
    e = hipMemcpyAsync(b->ctl, &c, sizeof(c), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev[0], b->stream);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev[1], b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return HY_OK;
}

hy_status hy_batch_autotune(hy_batch *b, double t_end, double cfl, int solver, int *best_bt, double *best_ms)
{
    if (!b) return fail(HY_EINVAL, "null batch");
    if (!(t_end > 0.0) || !std::isfinite(t_end)) return fail(HY_EINVAL, "t_end must be finite and > 0");
    if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(HY_EINVAL, "cfl must be finite and > 0");
    if (solver != HY_HLL && solver != HY_HLLC && solver != HY_HLLC_SWITCH) return fail(HY_EINVAL, "unknown solver");
    hy_status st = batch_order(b);
    if (st != HY_OK) return st;
    hy::BatchCtl c{};
    c.solver = solver == HY_HLLC_SWITCH ? HY_HLLC : solver;  // no transverse faces in 1D
    c.max_steps = kBatchMaxSteps;
    c.t_end = t_end;
    c.cfl = cfl;
    const size_t ubytes = sizeof(float) * 3 * (size_t)b->ntot;
    // the state is kept in the read-back scratch and restored before every
    // trial and at the end
    hipError_t e = hipMemcpyAsync(b->W, b->U, ubytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->ctl, &c, sizeof(c), hipMemcpyHostToDevice, b->stream);
    double bms = 1e300;
    int bbt = b->bt;
    std::vector<int> bts;
    bts.push_back(b->bt);  // the current size first, then the others
    for (int bt : {1024, 512, 256})
        if (bt != b->bt) bts.push_back(bt);
    for (int bt : bts) {
        const int nb = std::min(b->count, b->cus * hy::batch_blocks_per_cu(b->nmax, bt));
        if (e == hipSuccess) e = hipMemcpyAsync(b->U, b->W, ubytes, hipMemcpyDeviceToDevice, b->stream);
        if (e == hipSuccess) e = hy::launch_batch_reset(b->ctl, b->stream);
        if (e == hipSuccess) e = hipEventRecord(b->ev[0], b->stream);
        if (e == hipSuccess)
            e = hy::launch_batch(b->tubes, b->order, b->U, b->ntot, b->ctl, b->status, b->count, b->nmax, nb, bt,
                                 b->stream);
        if (e == hipSuccess) e = hipEventRecord(b->ev[1], b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b->ev[1]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->ev[0], b->ev[1]);
        if (e != hipSuccess) break;
        if (ms < (bt == b->bt ? bms : 0.98 * bms)) {  // the current size unless another is 2 % faster
            bms = ms;
            bbt = bt;
        }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(b->U, b->W, ubytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->status, 0, sizeof(hy::TubeStatus) * b->count, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch autotune");
    if (bbt != b->bt) {
        b->bt = bbt;
        b->nblocks = std::min(b->count, b->cus * hy::batch_blocks_per_cu(b->nmax, bbt));
        if (b->exec) {  // recaptured with the new workgroup size at the next run
            hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
    }
    if (best_bt) *best_bt = bbt;
    if (best_ms) *best_ms = bms;
    return HY_OK;
}

hy_status hy_batch_set_block(hy_batch *b, int bt)
{
    if (!b) return fail(HY_EINVAL, "null batch");
    if (!hy::batch_bt_supported(bt)) return fail(HY_EINVAL, "workgroup size must be 256, 512 or 1024");
    if (bt != b->bt) {
        b->bt = bt;
        b->nblocks = std::min(b->count, b->cus * hy::batch_blocks_per_cu(b->nmax, bt));
        if (b->exec) {
            hipError_t e = hipStreamSynchronize(b->stream);
            if (e != hipSuccess) return hip_fail(e, "batch sync");
            hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
    }
    return HY_OK;
}

hy_status hy_batch_get_block(hy_batch *b, int *bt)
{
    if (!b || !bt) return fail(HY_EINVAL, "null argument");
    *bt = b->bt;
    return HY_OK;
}

hy_status hy_batch_last_ms(hy_batch *b, double *ms)
{
    if (!b || !ms) return fail(HY_EINVAL, "null argument");
    hipError_t e = hipEventSynchronize(b->ev[1]);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, b->ev[0], b->ev[1]);
    if (e != hipSuccess) return hip_fail(e, "batch timing");
    *ms = t;
    return HY_OK;
}

hy_status hy_batch_get_state(hy_batch *b, int i, int kind, double *out)
{
    if (!b || !out) return fail(HY_EINVAL, "null argument");
    if (i < 0 || i >= b->count) return fail(HY_EINVAL, "tube index out of range");
    if (kind != HY_PRIMITIVE && kind != HY_CONSERVED) return fail(HY_EINVAL, "unknown state kind");
    const int64_t n = b->d[i].n[0];
    const float *src = b->U + b->off[i];
    hipError_t e = hipSuccess;
    if (kind == HY_PRIMITIVE) {
        e = hy::launch_cons_to_prim<float>(src, b->W + b->off[i], n, b->ntot, 1, (float)(b->d[i].gamma - 1.0), b->stream);
        src = b->W + b->off[i];
    }
    std::vector<float> st(3 * n);
    for (int v = 0; v < 3 && e == hipSuccess; ++v)
        e = hipMemcpyAsync(st.data() + v * n, src + v * b->ntot, sizeof(float) * n, hipMemcpyDeviceToHost, b->stream);
    hy::TubeStatus ts{};
    if (e == hipSuccess) e = hipMemcpyAsync(&ts, b->status + i, sizeof(ts), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "tube download");
    for (int64_t k = 0; k < 3 * n; ++k) out[k] = st[k];
    if (ts.err & 1) return fail(HY_ESTATE, "a kernel met rho <= 0, p <= 0 or a non-finite value in this tube");
    return HY_OK;
}

hy_status hy_batch_status(hy_batch *b, int i, int64_t *steps, double *t)
{
    if (!b || !steps || !t) return fail(HY_EINVAL, "null argument");
    if (i < 0 || i >= b->count) return fail(HY_EINVAL, "tube index out of range");
    hy::TubeStatus ts{};
    hipError_t e = hipMemcpyAsync(&ts, b->status + i, sizeof(ts), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "status download");
    *steps = ts.steps;
    *t = ts.t;
    if (ts.err & 1) return fail(HY_ESTATE, "a kernel met rho <= 0, p <= 0 or a non-finite value in this tube");
    if (ts.err & 2) return fail(HY_ESTATE, "the tube stopped before t_end (time step not > 0)");
    return HY_OK;
}

hy_status hy_batch_destroy(hy_batch *b)
{
    if (!b) return HY_OK;
    hipStreamSynchronize(b->stream);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->capture) hipStreamDestroy(b->capture);
    for (auto &ev : b->ev)
        if (ev) hipEventDestroy(ev);
    delete b;
    return HY_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Learned limiter: training data and trainer
// ------------------------------------------------------------------------
#include "hy_train.h"

namespace {

hy_status check_sample_patch(const hy_patch *p)
{
    if (!p) return fail(HY_EINVAL, "null patch");
    if (p->d.precision != 32) return fail(HY_EUNSUPPORTED, "training samples come from FP32 patches");
    for (int q = 0; q < p->d.ndim; ++q) {
        if (p->d.n[q] % 4 != 0 || p->d.n[q] < 20) return fail(HY_EINVAL, "sample patch needs n % 4 == 0 and n >= 20");
        if (p->d.bc[q][0] != HY_BC_PERIODIC) return fail(HY_EUNSUPPORTED, "sample patch must be periodic");
    }
    return HY_OK;
}

int64_t coarse_cells(const hy_patch *p)
{
    int64_t nc = 1;
    for (int q = 0; q < p->d.ndim; ++q) nc *= p->d.n[q] / 4;
    return nc;
}

}  // namespace

struct hy_trainer {
    hy::MlpDevice *m = nullptr;
    float *grad = nullptr, *m1 = nullptr, *m2 = nullptr, *partial = nullptr, *lpart = nullptr, *loss = nullptr;
    hipStream_t stream = nullptr;
    int step = 0;
};

extern "C" {

hy_status hy_lim_sample_count(const hy_patch *fine, int64_t *nsamples)
{
    hy_status st = check_sample_patch(fine);
    if (st != HY_OK) return st;
    if (!nsamples) return fail(HY_EINVAL, "null output");
    *nsamples = coarse_cells(fine) * (fine->d.ndim + 2) * fine->d.ndim;
    return HY_OK;
}

hy_status hy_lim_samples_scratch_bytes(const hy_patch *fine, size_t *bytes)
{
    hy_status st = check_sample_patch(fine);
    if (st != HY_OK) return st;
    if (!bytes) return fail(HY_EINVAL, "null output");
    const int nv = fine->d.ndim + 2;
    *bytes = sizeof(float) * (size_t)coarse_cells(fine) * (nv + (size_t)fine->d.ndim * nv * 4) + 256;
    return HY_OK;
}

hy_status hy_lim_make_samples(hy_patch *fine, void *dev_scratch, size_t scratch_bytes, float *x_dev, float *t_dev)
{
    hy_status st = check_sample_patch(fine);
    if (st != HY_OK) return st;
    if (!dev_scratch || !x_dev || !t_dev) return fail(HY_EINVAL, "null buffer");
    size_t need = 0;
    hy_lim_samples_scratch_bytes(fine, &need);
    if (scratch_bytes < need) return fail(HY_ENOMEM, "scratch too small");
    const int64_t nc = coarse_cells(fine);
    float *Wc = (float *)(((uintptr_t)dev_scratch + 255) & ~(uintptr_t)255);
    float *sub = Wc + (size_t)(fine->d.ndim + 2) * nc;
    const int nf[3] = {(int)fine->d.n[0], (int)fine->d.n[1], (int)fine->d.n[2]};
    const int ncd[3] = {nf[0] / 4, fine->d.ndim >= 2 ? nf[1] / 4 : 1, fine->d.ndim == 3 ? nf[2] / 4 : 1};
    hipError_t e = hy::launch_coarsen4((const float *)fine->A, fine->vstride, fine->d.ndim, nf,
                                       (float)(fine->d.gamma - 1.0), Wc, sub, fine->stream);
    if (e == hipSuccess) e = hy::launch_samples(Wc, sub, fine->d.ndim, ncd, x_dev, t_dev, fine->stream);
    if (e != hipSuccess) return hip_fail(e, "sample kernels");
    return HY_OK;
}

hy_status hy_lim_make_samples_noalloc(hy_patch *fine, float *x_dev, float *t_dev)
{
    hy_status st = check_sample_patch(fine);
    if (st != HY_OK) return st;
    if (!x_dev || !t_dev) return fail(HY_EINVAL, "null buffer");
    size_t need = 0;
    hy_lim_samples_scratch_bytes(fine, &need);
    if (need > hy::SAMPLES_STATIC_BYTES)
        return fail(HY_ENOMEM, "patch too large for the 64 MiB static sample staging");
    hipPointerAttribute_t attr{};
    hipError_t e = hipPointerGetAttributes(&attr, fine->A);
    if (e != hipSuccess) return hip_fail(e, "patch device");
    float *Wc = nullptr;
    e = hy::samples_static_scratch(attr.device, &Wc);
    if (e != hipSuccess) return hip_fail(e, "static staging address");
    const int64_t nc = coarse_cells(fine);
    float *sub = Wc + (size_t)(fine->d.ndim + 2) * nc;
    const int nf[3] = {(int)fine->d.n[0], (int)fine->d.n[1], (int)fine->d.n[2]};
    const int ncd[3] = {nf[0] / 4, fine->d.ndim >= 2 ? nf[1] / 4 : 1, fine->d.ndim == 3 ? nf[2] / 4 : 1};
    e = hy::launch_coarsen4((const float *)fine->A, fine->vstride, fine->d.ndim, nf, (float)(fine->d.gamma - 1.0), Wc,
                            sub, fine->stream);
    if (e == hipSuccess) e = hy::launch_samples(Wc, sub, fine->d.ndim, ncd, x_dev, t_dev, fine->stream);
    if (e != hipSuccess) return hip_fail(e, "sample kernels");
    return HY_OK;
}

hy_status hy_lim_slopes(hy_patch *p, float *out_dev)
{
    if (!p || !out_dev) return fail(HY_EINVAL, "null argument");
    if (p->d.limiter != HY_LIM_LEARNED || !p->mlp_set) return fail(HY_EINVAL, "patch has no learned limiter weights");
    hipError_t e = hy::launch_learned_slopes((const float *)p->A, out_dev, p->d.n, p->vstride, p->ncell, p->d.ndim,
                                             (float)(p->d.gamma - 1.0), p->d.bc, p->mlpimg, p->stream);
    if (e != hipSuccess) return hip_fail(e, "slope kernel");
    return HY_OK;
}

hy_status hy_trainer_workspace_bytes(size_t *bytes)
{
    if (!bytes) return fail(HY_EINVAL, "null output");
    *bytes = align_up(sizeof(hy::MlpDevice), 256) +
             sizeof(float) * ((size_t)hy::MLP_NPARAM * (3 + hy::TRAIN_BLOCKS) + hy::TRAIN_BLOCKS + 64) + 1024;
    return HY_OK;
}

hy_status hy_trainer_init(void *dev_workspace, size_t bytes, const float *params, void *hip_stream, hy_trainer **out)
{
    size_t need = 0;
    hy_trainer_workspace_bytes(&need);
    if (!dev_workspace || !params || !out) return fail(HY_EINVAL, "null argument");
    if (bytes < need) return fail(HY_ENOMEM, "workspace too small");
    hy_trainer *tr = new (std::nothrow) hy_trainer();
    if (!tr) return fail(HY_ENOMEM, "host allocation failed");
    char *base = (char *)(((uintptr_t)dev_workspace + 255) & ~(uintptr_t)255);
    tr->m = (hy::MlpDevice *)base;
    float *f = (float *)(base + align_up(sizeof(hy::MlpDevice), 256));
    tr->grad = f;
    tr->m1 = f + hy::MLP_NPARAM;
    tr->m2 = f + 2 * hy::MLP_NPARAM;
    tr->partial = f + 3 * hy::MLP_NPARAM;
    tr->lpart = tr->partial + (size_t)hy::MLP_NPARAM * hy::TRAIN_BLOCKS;
    tr->loss = tr->lpart + hy::TRAIN_BLOCKS;
    tr->stream = (hipStream_t)hip_stream;
    hy::MlpDevice host;
    hy::mlp_pack(params, &host);
    std::vector<float> zeros(2 * hy::MLP_NPARAM, 0.f);
    hipError_t e = hipMemcpyAsync(tr->m, &host, sizeof(host), hipMemcpyHostToDevice, tr->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(tr->m1, zeros.data(), sizeof(float) * 2 * hy::MLP_NPARAM, hipMemcpyHostToDevice, tr->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(tr->stream);
    if (e != hipSuccess) {
        delete tr;
        return hip_fail(e, "trainer init");
    }
    *out = tr;
    return HY_OK;
}

hy_status hy_trainer_step(hy_trainer *tr, const float *x_dev, const float *t_dev, const int32_t *idx_dev, int64_t batch,
                          float lr)
{
    if (!tr || !x_dev || !t_dev || !idx_dev) return fail(HY_EINVAL, "null argument");
    if (batch < 1 || !(lr > 0.f)) return fail(HY_EINVAL, "batch must be >= 1 and lr > 0");
    tr->step += 1;
    const hy::AdamStep ad = hy::adam_step(tr->m, tr->m1, tr->m2, lr, 0.9, 0.999, 1e-8f, tr->step);
    hipError_t e = hy::launch_train_grad(tr->m, x_dev, t_dev, idx_dev, batch, tr->partial, tr->lpart, hy::TRAIN_BLOCKS,
                                         tr->grad, tr->loss, ad, tr->stream);
    if (e != hipSuccess) return hip_fail(e, "training step");
    return HY_OK;
}

hy_status hy_trainer_gradient(hy_trainer *tr, const float *x_dev, const float *t_dev, const int32_t *idx_dev,
                              int64_t batch, float *grad_host, float *loss_host)
{
    if (!tr || !x_dev || !t_dev || !idx_dev || !grad_host || !loss_host) return fail(HY_EINVAL, "null argument");
    if (batch < 1) return fail(HY_EINVAL, "batch must be >= 1");
    hipError_t e = hy::launch_train_grad(tr->m, x_dev, t_dev, idx_dev, batch, tr->partial, tr->lpart, hy::TRAIN_BLOCKS,
                                         tr->grad, tr->loss, hy::AdamStep{}, tr->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(grad_host, tr->grad, sizeof(float) * hy::MLP_NPARAM, hipMemcpyDeviceToHost, tr->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(loss_host, tr->loss, sizeof(float), hipMemcpyDeviceToHost, tr->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(tr->stream);
    if (e != hipSuccess) return hip_fail(e, "gradient");
    return HY_OK;
}

hy_status hy_trainer_loss(hy_trainer *tr, float *loss_host)
{
    if (!tr || !loss_host) return fail(HY_EINVAL, "null argument");
    hipError_t e = hipMemcpyAsync(loss_host, tr->loss, sizeof(float), hipMemcpyDeviceToHost, tr->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(tr->stream);
    if (e != hipSuccess) return hip_fail(e, "loss");
    return HY_OK;
}

hy_status hy_trainer_get_params(hy_trainer *tr, float *params_host)
{
    if (!tr || !params_host) return fail(HY_EINVAL, "null argument");
    hipError_t e = hipMemcpyAsync(params_host, tr->m, sizeof(float) * hy::MLP_NPARAM, hipMemcpyDeviceToHost, tr->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(tr->stream);
    if (e != hipSuccess) return hip_fail(e, "parameter download");
    return HY_OK;
}

hy_status hy_mlp_eval(hy_trainer *tr, const float *x_dev, float *y_dev, int64_t batch)
{
    if (!tr || !x_dev || !y_dev) return fail(HY_EINVAL, "null argument");
    if (batch < 0) return fail(HY_EINVAL, "batch must be >= 0");
    hipError_t e = hy::launch_mlp_forward(tr->m, x_dev, y_dev, batch, tr->stream);
    if (e != hipSuccess) return hip_fail(e, "network evaluation");
    return HY_OK;
}

hy_status hy_trainer_destroy(hy_trainer *tr)
{
    if (!tr) return HY_OK;
    hipStreamSynchronize(tr->stream);
    delete tr;
    return HY_OK;
}

}  // extern "C"

// ================================================ fixed multilevel refinement
//
// Host recursion of Algs. Evolve / EvolveLevel / StepLevel over nested levels.
// Level 0 is an ordinary patch with the physical boundaries; a refined level
// is a patch over its cells plus a two-cell exterior, stepped by the stage
// kernels' padded mode (interior updated, exterior read as ghost cells; its
// boundary kinds go unused), the exterior written by prolongation into both
// the state and the stage state before each step.  The levels' times and
// steps live in device clocks, so a global step is a fixed launch sequence:
// captured once into a HIP graph and replayed; the host waits once, at the
// end, for the error latches and the coarse step.
#include "hy_fmr.h"

// A job for fmr_ride (host side, precision-free): the prolongation of a
// padded level's exterior from its parent (fine != null; arguments of
// hy::launch_prolong) and the clock updates ck.
struct FmrRide {
    void *fine, *fine2;
    hy::Grid fg;
    const void *parent;
    hy::Grid pg;
    hy::Box pb;
    int ndim;
    double gm1;
    hy::ClockOps ck;
};

template <typename T>
hy::RideJob<T> ride_job(const FmrRide &r)
{
    if (r.fine)
        return hy::prolong_job<T>((T *)r.fine, (T *)r.fine2, r.fg, (const T *)r.parent, r.pg, r.pb, r.ndim, (T)r.gm1,
                                  r.ck);
    hy::RideJob<T> j{};
    j.ck = r.ck;
    return j;
}

struct hy_fmr {
    hy_fmr_desc d;
    int nlev = 0, nv = 0;
    hipStream_t stream = nullptr;
    struct Level {
        hy_patch *p = nullptr;
        int64_t n[3] = {1, 1, 1};  // interior cells
        int off = 0;               // interior offset per active dimension (0 or NG)
        hy::Grid g{};
        hy::Box own{};             // interior, array coordinates
        hy::Box child{};           // cells the next level refines, array coordinates (n[0] = 0: none)
        double idq[3] = {0, 0, 0};
        double dv = 1.0;
        double *own_acc[3][2] = {};     // boundary fluxes over the last two steps (for the parent)
        double *coarse_acc[3][2] = {};  // this level's fluxes at the child's faces over one step
        double *partials = nullptr;     // leaf totals, rows x 5
        int64_t rows = 0;
        bool prov = false;       // the provisional half-step result sits in the patch's stage buffer
        bool own_fresh = false;  // own_acc holds nothing yet: the next write assigns
    } lev[HY_FMR_MAXLEV];
    unsigned long long *rate = nullptr;
    hy::FmrClock *clock = nullptr;
    int pending_advance = -1;  // level whose clock advance rides on the next clock launch
    // the last launch of a level's step (the second stage of the deepest
    // level, else the coarse/fine replacement and restriction from its
    // child), held back so that the parent's prolongation or clock update
    // that comes next can ride on it (fmr_ride); or a refined level's
    // provisional first stage, on which the deepest level's prolongation can
    // ride unless the deepest level is its child; launched with ride == null
    // otherwise (fmr_flush)
    int held_level = -1;
    bool held_prov = false;
    std::function<hipError_t(const FmrRide *ride)> held;
    int solver = HY_HLLC;
    double cfl = 0.4, dt_fixed = 0.0;
    // the launches of one global step, captured once per (solver, cfl,
    // dt_fixed) on a private stream and replayed on the caller's
    bool use_graph = true;
    hipStream_t capture = nullptr;
    hipGraphExec_t exec = nullptr;
    int g_solver = -1;
    double g_cfl = 0.0, g_dt_fixed = 0.0;
};

namespace {

struct FmrLayout {
    hy_patch_desc desc[HY_FMR_MAXLEV];
    size_t patch[HY_FMR_MAXLEV], own[HY_FMR_MAXLEV][3], coarse[HY_FMR_MAXLEV][3], partials[HY_FMR_MAXLEV];
    size_t patch_bytes[HY_FMR_MAXLEV], own_bytes[HY_FMR_MAXLEV][3], coarse_bytes[HY_FMR_MAXLEV][3];
    size_t rate, clock, total;
};

int64_t transverse(const int64_t n[3], int q) { return n[(q + 1) % 3] * n[(q + 2) % 3]; }

hy_status fmr_layout(const hy_fmr_desc *d, FmrLayout *L)
{
    if (!d) return fail(HY_EINVAL, "null descriptor");
    hy_status st = check_desc(&d->base);
    if (st != HY_OK) return st;
    if (d->nlev < 1 || d->nlev > HY_FMR_MAXLEV) return fail(HY_EINVAL, "nlev must lie in 1 .. HY_FMR_MAXLEV");
    if (d->base.limiter != HY_LIM_THETA) return fail(HY_EUNSUPPORTED, "multilevel runs take the theta limiter");
    const int nd = d->base.ndim, nv = nd + 2;
    int64_t n[3] = {d->base.n[0], d->base.n[1], d->base.n[2]};
    size_t o = 0;
    for (int l = 0; l < d->nlev; ++l) {
        hy_patch_desc pd = d->base;
        if (l > 0) {
            const hy_patch_desc &pp = L->desc[l - 1];
            const int poff = l > 1 ? hy::FMR_NG : 0;
            for (int q = 0; q < 3; ++q) {
                const int64_t lo = d->box_lo[l][q], bn = d->box_n[l][q];
                if (q < nd) {
                    if (bn < 1 || lo < hy::FMR_NG || lo + bn > n[q] - hy::FMR_NG)
                        return fail(HY_EINVAL, "a refined box must keep two parent cells from its parent's edge");
                    const double dqp = (pp.hi[q] - pp.lo[q]) / (double)pp.n[q];
                    const double dq = 0.5 * dqp;
                    n[q] = 2 * bn;
                    pd.n[q] = n[q] + 2 * hy::FMR_NG;
                    pd.lo[q] = pp.lo[q] + (double)(lo + poff) * dqp - hy::FMR_NG * dq;
                    pd.hi[q] = pd.lo[q] + (double)pd.n[q] * dq;
                    pd.bc[q][0] = pd.bc[q][1] = HY_BC_OUTFLOW;
                } else if (lo != 0 || bn != 1) {
                    return fail(HY_EINVAL, "unused dimensions take box_lo 0 and box_n 1");
                }
            }
            st = check_desc(&pd);
            if (st != HY_OK) return st;
        }
        L->desc[l] = pd;
        L->patch[l] = o;
        L->patch_bytes[l] = layout(pd).total;
        o = align_up(o + L->patch_bytes[l], 256);
        for (int q = 0; q < 3; ++q) {
            L->own_bytes[l][q] = 0;
            L->coarse_bytes[l][q] = 0;
            if (q >= nd) continue;
            if (l > 0) {
                L->own[l][q] = o;
                L->own_bytes[l][q] = sizeof(double) * nv * (size_t)transverse(n, q);
                o = align_up(o + 2 * L->own_bytes[l][q], 256);
            }
            if (l + 1 < d->nlev) {
                L->coarse[l][q] = o;
                L->coarse_bytes[l][q] = sizeof(double) * nv * (size_t)transverse(d->box_n[l + 1], q);
                o = align_up(o + 2 * L->coarse_bytes[l][q], 256);
            }
        }
        L->partials[l] = o;
        o = align_up(o + sizeof(double) * 5 * (size_t)(n[1] * n[2]), 256);
    }
    L->rate = o;
    o = align_up(o + sizeof(unsigned long long) * hy::FMR_RATE_SLOTS, 256);
    L->clock = o;
    o = align_up(o + sizeof(hy::FmrClock) * HY_FMR_MAXLEV, 256);
    L->total = o + 256;
    return HY_OK;
}

// Launches the held launch as it is.  Every other launch of the multilevel
// step goes after this.
hipError_t fmr_flush(hy_fmr *f)
{
    if (!f->held) return hipSuccess;
    auto fn = std::move(f->held);
    f->held = nullptr;
    f->held_level = -1;
    return fn(nullptr);
}

void fmr_hold(hy_fmr *f, int level, std::function<hipError_t(const FmrRide *)> fn, bool prov = false)
{
    f->held = std::move(fn);
    f->held_level = level;
    f->held_prov = prov;
}

// Launches job r (the parent's prolongation and/or clock updates of level l)
// riding on the held launch when that is the end of level l + 1's step (it
// then touches nothing the job does: the held launch writes level l + 1 (its
// state, its own boundary fluxes, or the child's restriction into it) and
// reads only its own step from the clocks, the job writes level l's
// exterior, reads level l - 1, and updates the clocks of level l and the
// advance of level l + 1's time); else after flushing it, in a launch of its
// own.  Returns false in *rode when it did not ride.
hipError_t fmr_ride(hy_fmr *f, int l, const FmrRide &r, bool *rode)
{
    *rode = false;
    // (a provisional first stage of level m writes level m's stage state and
    // reads level m and its clock; the deepest level's prolongation reads its
    // parent's state and its own rate words and writes its exterior and
    // clock: independent unless m is the parent)
    const bool ok = f->held_prov ? (l == f->nlev - 1 && f->held_level <= l - 2 && r.fine != nullptr)
                                 : f->held_level == l + 1;
    if (f->held && ok) {
        auto fn = std::move(f->held);
        f->held = nullptr;
        f->held_level = -1;
        *rode = true;
        return fn(&r);
    }
    return fmr_flush(f);
}

// A clock update on the stream; a pending advance of a level's time goes
// first in the same launch.
hipError_t fmr_clock(hy_fmr *f, int op, int l, unsigned long long *rate = nullptr)
{
    const int pre = f->pending_advance;
    f->pending_advance = -1;
    FmrRide r{};
    r.ck = {f->clock, pre >= 0 ? hy::CLOCK_ADVANCE : -1, pre, op, l, f->nlev, rate ? rate : f->rate, f->cfl, f->dt_fixed};
    bool rode = false;
    hipError_t e = op >= 0 || pre >= 0 ? fmr_ride(f, l, r, &rode) : fmr_flush(f);
    if (e != hipSuccess || rode) return e;
    return hy::launch_clock(f->clock, r.ck.op0, r.ck.l0, r.ck.op1, r.ck.l1, f->nlev, r.ck.rate, f->cfl, f->dt_fixed,
                            f->stream);
}

// Level l's time advances by its step; the update joins the next clock launch
// (nothing reads the time before then).
hipError_t fmr_defer_advance(hy_fmr *f, int l)
{
    hipError_t e = hipSuccess;
    if (f->pending_advance >= 0) e = fmr_clock(f, -1, 0);
    f->pending_advance = l;
    return e;
}

template <typename T> T *arrA(hy_fmr::Level &L) { return (T *)L.p->A; }
template <typename T> T *arrB(hy_fmr::Level &L) { return (T *)L.p->B; }

// Prolongation into level l's exterior; the pending clock advance and the
// clock update op (on level lop; op < 0: none) ride on the same launch.
template <typename T>
hipError_t fmr_prolong(hy_fmr *f, int l, int op = -1, int lop = 0, unsigned long long *rate = nullptr)
{
    hy_fmr::Level &L = f->lev[l], &P = f->lev[l - 1];
    hy::Box pb{};
    for (int q = 0; q < 3; ++q) {
        pb.lo[q] = (int)(f->d.box_lo[l][q] + (q < f->d.base.ndim ? P.off : 0));
        pb.n[q] = (int)f->d.box_n[l][q];
    }
    const T *src = P.prov ? arrB<T>(P) : arrA<T>(P);
    const double g = f->d.base.gamma;
    // the exterior of both the level's state and its stage state: the stages
    // update interiors only, so the exterior stays fixed through the step
    hy::ClockOps ck{};
    const int pre = f->pending_advance;
    f->pending_advance = -1;
    if (pre >= 0 || op >= 0)
        ck = {f->clock, pre >= 0 ? hy::CLOCK_ADVANCE : -1, pre, op, lop, f->nlev, rate ? rate : f->rate, f->cfl,
              f->dt_fixed};
    // rides on the end of the child's step when that was the last launch
    // (never for the deepest level, whose exterior comes from the parent's
    // state of the launches just before)
    const FmrRide r{arrA<T>(L), arrB<T>(L), L.g, src, P.g, pb, f->d.base.ndim, g - 1.0, ck};
    bool rode = false;
    hipError_t e = fmr_ride(f, l, r, &rode);
    if (e != hipSuccess || rode) return e;
    return hy::launch_prolong<T>(arrA<T>(L), arrB<T>(L), L.g, src, P.g, pb, f->d.base.ndim, (T)g, (T)(g - 1.0), ck,
                                 f->stream);
}

// Stepper(l)%Step with the level's step from its device clock (dt, or dtp for
// the provisional half-step).
template <typename T>
hipError_t fmr_level_step(hy_fmr *f, int l, bool provisional)
{
    hy_fmr::Level &L = f->lev[l];
    hy_patch *p = L.p;
    hipError_t e = fmr_flush(f);
    if (e != hipSuccess) return e;
    if (provisional) {
        p->dt_dev = &f->clock[l].dtp;
        if (l > 0) {
            // a refined parent updates only the cells the child's
            // prolongation reads: the child box grown by two cells (a view of
            // the padded array; the box keeps two cells from the level's edge,
            // so the view's ghosts lie inside the array)
            hy::StageArgs<T> a = stage_args<T>(p, 1, hy::DT_PTR, 0.0, 0.0, 0.0);
            for (int q = 0; q < p->d.ndim; ++q) {
                a.n[q] = f->d.box_n[l + 1][q] + 4;
                a.voff[q] = (int)f->d.box_lo[l + 1][q];  // NG + (box_lo - 2) in storage
            }
            // held: the deepest level's prolongation may come next and ride on it
            const int nd = p->d.ndim, solver = f->solver;
            const hy::LaunchCfg cfg = p->cfg;
            hipStream_t st = p->stream;
            fmr_hold(f, l, [a, nd, solver, cfg, st](const FmrRide *r) {
                hy::StageArgs<T> b = a;
                if (r) b.ride = ride_job<T>(*r);
                return hy::launch_stage<T>(nd, solver, 1, hy::LIM_THETA_PADDED, cfg, b, st);
            }, true);
        } else {
            e = run_stage<T>(p, f->solver, 1, hy::DT_PTR, 0.0, 0.0, 0.0);
        }
        L.prov = true;
        return e;
    }
    const int nd = f->d.base.ndim;
    const bool child = l + 1 < f->nlev;
    const double g = f->d.base.gamma;
    const double *dt = &f->clock[l].dt;
    p->dt_dev = dt;
    const T gamma = (T)g, gm1 = (T)(g - 1.0), igm1 = (T)(1.0 / (g - 1.0)), theta = (T)f->d.base.theta;
    // the fluxes through the child's faces (replaced later) and through this
    // level's own boundary (handed to the parent), from each stage's input
    hy::Box boxes[2];
    double *const(*accs[2])[2] = {nullptr, nullptr};
    int nbox = 0, assign[2] = {0, 0}, kc = -1, ko = -1;
    if (child) {
        boxes[nbox] = L.child;
        kc = nbox;
        accs[nbox++] = L.coarse_acc;
    }
    if (l > 0) {
        boxes[nbox] = L.own;
        ko = nbox;
        accs[nbox++] = L.own_acc;
    }
    double *acc[2][3][2];
    for (int k = 0; k < nbox; ++k)
        for (int q = 0; q < 3; ++q)
            for (int s = 0; s < 2; ++s) acc[k][q][s] = accs[k][q][s];
    for (int stage = 1; stage <= 2; ++stage) {
        const T *u = stage == 1 ? arrA<T>(L) : arrB<T>(L);
        if (nbox > 0) {
            // the child-face fluxes start afresh each step; the boundary
            // fluxes afresh after the parent has consumed them
            if (kc >= 0) assign[kc] = stage == 1;
            if (ko >= 0) assign[ko] = stage == 1 && L.own_fresh;
            if (l > 0) {
                // a padded level's stage launch computes the box fluxes too
                hy::StageArgs<T> a = stage_args<T>(p, stage, hy::DT_PTR, 0.0, 0.0, 0.0);
                a.bf.nbox = nbox;
                for (int k = 0; k < nbox; ++k) {
                    a.bf.b[k] = boxes[k];
                    a.bf.assign[k] = assign[k];
                    for (int q = 0; q < 3; ++q)
                        for (int sd = 0; sd < 2; ++sd) a.bf.acc[k][q][sd] = acc[k][q][sd];
                }
                if (stage == 2 && !child) {
                    // the deepest level's second stage ends its step: held
                    // for the parent's prolongation or clock update to ride on
                    const int solver = f->solver;
                    const hy::LaunchCfg cfg = p->cfg;
                    hipStream_t st = p->stream;
                    fmr_hold(f, l, [a, nd, solver, cfg, st](const FmrRide *r) {
                        hy::StageArgs<T> b = a;
                        if (r) b.ride = ride_job<T>(*r);
                        return hy::launch_stage<T>(nd, solver, 2, hy::LIM_THETA_PADDED, cfg, b, st);
                    });
                } else {
                    e = hy::launch_stage<T>(nd, f->solver, stage, hy::LIM_THETA_PADDED, p->cfg, a, p->stream);
                    if (e != hipSuccess) return e;
                }
                L.own_fresh = false;
                continue;
            }
            e = hy::launch_box_flux<T>(u, L.g, nbox, boxes, acc, assign, nd, f->solver, gamma, gm1, igm1, theta, dt,
                                       f->stream);
            if (e != hipSuccess) return e;
            L.own_fresh = false;
        }
        e = run_stage<T>(p, f->solver, stage, hy::DT_PTR, 0.0, 0.0, 0.0);
        if (e != hipSuccess) return e;
    }
    p->parity ^= 1;
    return e;
}

template <typename T>
hy_status fmr_step_level(hy_fmr *f, int l);

template <typename T>
hy_status fmr_evolve_level(hy_fmr *f, int l)
{
    if (l >= f->nlev) return HY_OK;
    hy_status st = fmr_step_level<T>(f, l);
    if (st != HY_OK || l == 0) return st;
    // the provisional step of the parent: its exterior (if it has a parent),
    // its step (the child's first), then its first stage
    hipError_t e = l - 1 > 0 ? fmr_prolong<T>(f, l - 1, hy::CLOCK_PROVISIONAL, l - 1)
                             : fmr_clock(f, hy::CLOCK_PROVISIONAL, l - 1);
    if (e == hipSuccess) e = fmr_level_step<T>(f, l - 1, true);
    if (e != hipSuccess) return hip_fail(e, "provisional coarse step");
    st = fmr_step_level<T>(f, l);
    f->lev[l - 1].prov = false;
    return st;
}

template <typename T>
hy_status fmr_step_level(hy_fmr *f, int l)
{
    hy_fmr::Level &L = f->lev[l];
    const int nd = f->d.base.ndim;
    hipError_t e;
    if (l + 1 < f->nlev) {
        f->lev[l + 1].own_fresh = true;  // the child's boundary fluxes over its next two steps
        hy_status st = fmr_evolve_level<T>(f, l + 1);
        if (st != HY_OK) return st;
    }
    // Alg. StepLevel's time step: the CFL step at the deepest level, else
    // the span of the child's two steps; on a refined level the clock update
    // rides on the prolongation of its exterior
    const bool deepest = l == f->nlev - 1;
    if (l > 0) {
        // the deepest refined level's rate is the one its last second stage
        // (or hy_set_state) left in its control block: its stages cover its
        // interior only, and nothing else changes it between its steps; its
        // 2^l steps per global step leave the parity slot where a replay of
        // the captured step expects it
        static_assert(hy::FMR_RATE_SLOTS == hy::RATE_SLOTS, "rate words");
        e = deepest ? fmr_prolong<T>(f, l, hy::CLOCK_DEEPEST_KEEP, l, &L.p->ctl->rate[L.p->parity][0])
                    : fmr_prolong<T>(f, l, hy::CLOCK_COARSE, l);
    } else if (deepest) {  // one level: a rate pass over it
        e = fmr_flush(f);
        if (e == hipSuccess && !(f->dt_fixed > 0.0)) {
            const double g = f->d.base.gamma;
            e = hy::launch_box_rate<T>(arrA<T>(L), L.g, L.own, nd, (T)g, (T)(g - 1.0), L.idq, f->rate, f->stream);
        }
        if (e == hipSuccess) e = fmr_clock(f, hy::CLOCK_DEEPEST, l);
    } else {
        e = fmr_clock(f, hy::CLOCK_COARSE, l);
    }
    if (e != hipSuccess) return hip_fail(e, "prolongation and time step");
    e = fmr_level_step<T>(f, l, false);
    if (e == hipSuccess && l + 1 < f->nlev) {
        // the coarse/fine flux replacement and the restriction of the child
        hy_fmr::Level &C = f->lev[l + 1];
        const double *c[3][2], *fa[3][2];
        for (int q = 0; q < 3; ++q)
            for (int s = 0; s < 2; ++s) {
                c[q][s] = L.coarse_acc[q][s];
                fa[q][s] = C.own_acc[q][s];
            }
        // held: it ends this level's step, and the parent's prolongation or
        // clock update (or the coarse level's final clock advance) that
        // comes next can ride on it
        struct Args {
            T *u;
            hy::Grid g, cg;
            hy::Box child;
            const double *c[3][2], *fa[3][2];
            double idq[3];
            const T *uc;
        } ra{arrA<T>(L), L.g, C.g, L.child, {}, {}, {L.idq[0], L.idq[1], L.idq[2]}, arrA<T>(C)};
        for (int q = 0; q < 3; ++q)
            for (int sd = 0; sd < 2; ++sd) {
                ra.c[q][sd] = c[q][sd];
                ra.fa[q][sd] = fa[q][sd];
            }
        hipStream_t st = f->stream;
        e = fmr_flush(f);
        if (e == hipSuccess)
            fmr_hold(f, l, [ra, nd, st](const FmrRide *r) {
                hy::RideJob<T> j{};
                if (r) j = ride_job<T>(*r);
                return hy::launch_reflux_restrict<T>(ra.u, ra.g, ra.child, nd, ra.c, ra.fa, ra.idq, ra.uc, ra.cg,
                                                     r ? &j : nullptr, st);
            });
    }
    if (e == hipSuccess) e = fmr_defer_advance(f, l);
    if (e != hipSuccess) return hip_fail(e, "level step");
    return HY_OK;
}

// Enqueues one global step on stream s (every level's launches go there).
hy_status fmr_enqueue(hy_fmr *f, hipStream_t s)
{
    f->stream = s;
    for (int l = 0; l < f->nlev; ++l) {
        f->lev[l].p->stream = s;
        f->lev[l].prov = false;
    }
    f->pending_advance = -1;
    f->held = nullptr;
    f->held_level = -1;
    hipError_t e = fmr_clock(f, hy::CLOCK_RESET, 0);
    if (e != hipSuccess) return hip_fail(e, "clock reset");
    hy_status st = f->d.base.precision == 64 ? fmr_evolve_level<double>(f, 0) : fmr_evolve_level<float>(f, 0);
    if (st != HY_OK) {
        f->held = nullptr;
        f->held_level = -1;
        return st;
    }
    // the coarse level's final advance, riding on its restriction from
    // level 1 when that was the last launch
    const int pre = f->pending_advance;
    f->pending_advance = -1;
    if (pre >= 0 && f->held && !f->held_prov && f->held_level == 0) {
        FmrRide r{};
        r.ck = {f->clock, hy::CLOCK_ADVANCE, pre, -1, 0, f->nlev, f->rate, f->cfl, f->dt_fixed};
        auto fn = std::move(f->held);
        f->held = nullptr;
        f->held_level = -1;
        e = fn(&r);
    } else {
        e = fmr_flush(f);
        if (e == hipSuccess && pre >= 0)
            e = hy::launch_clock(f->clock, hy::CLOCK_ADVANCE, pre, -1, 0, f->nlev, f->rate, f->cfl, f->dt_fixed,
                                 f->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "clock advance");
    return HY_OK;
}

void fmr_drop_graph(hy_fmr *f)
{
    if (f->exec) (void)hipGraphExecDestroy(f->exec);
    f->exec = nullptr;
}

// Captures the global step's launches into f->exec (none of them is a
// memset or a host wait).
hy_status fmr_capture(hy_fmr *f, hipStream_t caller)
{
    fmr_drop_graph(f);
    hipError_t e = hipSuccess;
    if (!f->capture) e = hipStreamCreateWithFlags(&f->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(f->capture, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    hy_status st = fmr_enqueue(f, f->capture);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(f->capture, &g);
    // every later launch outside the graph goes to the caller's stream again
    f->stream = caller;
    for (int l = 0; l < f->nlev; ++l) f->lev[l].p->stream = caller;
    if (st != HY_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&f->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        f->exec = nullptr;
        return hip_fail(e, "graph capture");
    }
    f->g_solver = f->solver;
    f->g_cfl = f->cfl;
    f->g_dt_fixed = f->dt_fixed;
    return HY_OK;
}

hy_status fmr_check_level(hy_fmr *f, int level)
{
    if (!f) return fail(HY_EINVAL, "null handle");
    if (level < 0 || level >= f->nlev) return fail(HY_EINVAL, "no such level");
    return HY_OK;
}

}  // namespace

extern "C" {

hy_status hy_fmr_workspace_bytes(const hy_fmr_desc *d, size_t *bytes)
{
    if (!bytes) return fail(HY_EINVAL, "null output");
    FmrLayout L;
    hy_status st = fmr_layout(d, &L);
    if (st != HY_OK) return st;
    *bytes = L.total;
    return HY_OK;
}

hy_status hy_fmr_init(const hy_fmr_desc *d, void *dev_workspace, size_t bytes, void *hip_stream, hy_fmr **out)
{
    FmrLayout L;
    hy_status st = fmr_layout(d, &L);
    if (st != HY_OK) return st;
    if (!out || !dev_workspace) return fail(HY_EINVAL, "null workspace or output handle");
    if (bytes < L.total) return fail(HY_ENOMEM, "workspace too small");
    hy_fmr *f = new (std::nothrow) hy_fmr();
    if (!f) return fail(HY_ENOMEM, "host allocation failed");
    f->d = *d;
    f->nlev = d->nlev;
    f->nv = d->base.ndim + 2;
    f->stream = (hipStream_t)hip_stream;
    const int nd = d->base.ndim;
    char *base = (char *)(((uintptr_t)dev_workspace + 255) & ~(uintptr_t)255);
    for (int l = 0; l < f->nlev; ++l) {
        hy_fmr::Level &V = f->lev[l];
        st = hy_init_patch(&L.desc[l], base + L.patch[l], L.patch_bytes[l], hip_stream, &V.p);
        if (st != HY_OK) {
            hy_fmr_destroy(f);
            return st;
        }
        V.off = l > 0 ? hy::FMR_NG : 0;
        V.g.vs = V.p->vstride;
        if (l > 0) {
            V.p->padded = true;
            for (int q = 0; q < 3; ++q) V.p->inner[q] = q < nd ? L.desc[l].n[q] - 2 * hy::FMR_NG : 1;
            pick_config(V.p);
        }
        V.dv = 1.0;
        for (int q = 0; q < 3; ++q) {
            const bool act = q < nd;
            V.g.m[q] = (int)L.desc[l].n[q];
            V.n[q] = act ? L.desc[l].n[q] - 2 * V.off : 1;
            V.own.lo[q] = act ? V.off : 0;
            V.own.n[q] = (int)V.n[q];
            V.idq[q] = act ? (double)L.desc[l].n[q] / (L.desc[l].hi[q] - L.desc[l].lo[q]) : 0.0;
            if (act) V.dv /= V.idq[q];
            if (l + 1 < f->nlev) {
                V.child.lo[q] = (int)(d->box_lo[l + 1][q] + (act ? V.off : 0));
                V.child.n[q] = (int)d->box_n[l + 1][q];
            }
            if (act) {
                if (l > 0) {
                    V.own_acc[q][0] = (double *)(base + L.own[l][q]);
                    V.own_acc[q][1] = (double *)(base + L.own[l][q] + L.own_bytes[l][q]);
                }
                if (l + 1 < f->nlev) {
                    V.coarse_acc[q][0] = (double *)(base + L.coarse[l][q]);
                    V.coarse_acc[q][1] = (double *)(base + L.coarse[l][q] + L.coarse_bytes[l][q]);
                }
            }
        }
        V.partials = (double *)(base + L.partials[l]);
        V.rows = V.n[1] * V.n[2];
    }
    f->rate = (unsigned long long *)(base + L.rate);
    f->clock = (hy::FmrClock *)(base + L.clock);
    *out = f;
    return HY_OK;
}

hy_status hy_fmr_set_state(hy_fmr *f, int level, int kind, const double *host)
{
    hy_status st = fmr_check_level(f, level);
    if (st != HY_OK) return st;
    if (!host) return fail(HY_EINVAL, "null argument");
    hy_fmr::Level &V = f->lev[level];
    if (V.off == 0) return hy_set_state(V.p, kind, host);
    // a refined level's array is padded: the exterior starts as a copy of the
    // nearest interior cell (prolongation replaces it before it is used)
    const int nd = f->d.base.ndim;
    const int64_t N = V.n[0] * V.n[1] * V.n[2];
    const int64_t M = (int64_t)V.g.m[0] * V.g.m[1] * V.g.m[2];
    std::vector<double> pad((size_t)(f->nv * M));
    for (int64_t k = 0; k < V.g.m[2]; ++k)
        for (int64_t j = 0; j < V.g.m[1]; ++j)
            for (int64_t i = 0; i < V.g.m[0]; ++i) {
                const int64_t c3[3] = {i, j, k};
                int64_t s3[3];
                for (int q = 0; q < 3; ++q)
                    s3[q] = q < nd ? std::min(std::max(c3[q] - V.off, (int64_t)0), V.n[q] - 1) : 0;
                const int64_t src = (s3[2] * V.n[1] + s3[1]) * V.n[0] + s3[0];
                const int64_t dst = (k * V.g.m[1] + j) * V.g.m[0] + i;
                for (int v = 0; v < f->nv; ++v) pad[(size_t)(v * M + dst)] = host[v * N + src];
            }
    return hy_set_state(V.p, kind, pad.data());
}

hy_status hy_fmr_get_state(hy_fmr *f, int level, int kind, double *out)
{
    hy_status st = fmr_check_level(f, level);
    if (st != HY_OK) return st;
    if (!out) return fail(HY_EINVAL, "null argument");
    hy_fmr::Level &V = f->lev[level];
    if (V.off == 0) return hy_get_state(V.p, kind, out);
    const int nd = f->d.base.ndim;
    const int64_t N = V.n[0] * V.n[1] * V.n[2];
    const int64_t M = (int64_t)V.g.m[0] * V.g.m[1] * V.g.m[2];
    std::vector<double> pad((size_t)(f->nv * M));
    st = hy_get_state(V.p, kind, pad.data());
    if (st != HY_OK && st != HY_ESTATE) return st;
    for (int64_t k = 0; k < V.n[2]; ++k)
        for (int64_t j = 0; j < V.n[1]; ++j)
            for (int64_t i = 0; i < V.n[0]; ++i) {
                const int64_t src = ((k + (nd > 2 ? V.off : 0)) * V.g.m[1] + j + (nd > 1 ? V.off : 0)) * V.g.m[0] + i + V.off;
                const int64_t dst = (k * V.n[1] + j) * V.n[0] + i;
                for (int v = 0; v < f->nv; ++v) out[v * N + dst] = pad[(size_t)(v * M + src)];
            }
    return st;
}

hy_status hy_fmr_set_graph(hy_fmr *f, int on)
{
    if (!f) return fail(HY_EINVAL, "null handle");
    f->use_graph = on != 0;
    if (!f->use_graph) fmr_drop_graph(f);
    return HY_OK;
}

hy_status hy_fmr_step(hy_fmr *f, double cfl, double dt_fixed, int solver, double *dt_out)
{
    if (!f) return fail(HY_EINVAL, "null handle");
    if (solver != HY_HLL && solver != HY_HLLC) return fail(HY_EINVAL, "multilevel steps take HY_HLL or HY_HLLC");
    if (!(dt_fixed > 0.0) && !(cfl > 0.0 && std::isfinite(cfl))) return fail(HY_EINVAL, "need cfl > 0 or dt_fixed > 0");
    if (dt_fixed > 0.0 && !std::isfinite(dt_fixed)) return fail(HY_EINVAL, "dt_fixed must be finite");
    f->solver = solver;
    f->cfl = cfl;
    f->dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
    hipStream_t caller = f->stream;
    hy_status st;
    hipError_t e;
    if (f->use_graph) {
        if (!f->exec || f->g_solver != f->solver || f->g_cfl != f->cfl || f->g_dt_fixed != f->dt_fixed) {
            st = fmr_capture(f, caller);
            if (st != HY_OK) return st;
        }
        e = hipGraphLaunch(f->exec, caller);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
    } else {
        st = fmr_enqueue(f, caller);
        if (st != HY_OK) return st;
    }
    hy::FmrClock c0;
    e = hipMemcpyAsync(&c0, f->clock, sizeof(c0), hipMemcpyDeviceToHost, f->stream);
    if (e != hipSuccess) return hip_fail(e, "clock read");
    for (int l = 0; l < f->nlev; ++l) {
        hy::DevCtl c;
        st = read_ctl(f->lev[l].p, &c);  // synchronises the stream
        if (st != HY_OK) return st;
        if (c.err) return fail(HY_ESTATE, "a kernel met rho <= 0, p <= 0 or a non-finite value");
    }
    if (!(c0.t > 0.0) || !std::isfinite(c0.t))
        return fail(HY_ESTATE, "the deepest level's CFL step is not positive and finite");
    if (dt_out) *dt_out = c0.t;
    return HY_OK;
}

hy_status hy_fmr_conserved_totals(hy_fmr *f, double out[5])
{
    if (!f || !out) return fail(HY_EINVAL, "null argument");
    for (int k = 0; k < 5; ++k) out[k] = 0.0;
    const int nd = f->d.base.ndim;
    for (int l = 0; l < f->nlev; ++l) {
        hy_fmr::Level &V = f->lev[l];
        hy::Box hole{};
        if (l + 1 < f->nlev) hole = V.child;
        hipError_t e;
        if (f->d.base.precision == 64)
            e = hy::launch_leaf_totals<double>((const double *)V.p->A, V.g, V.own, hole, nd, V.dv, V.partials, f->stream);
        else
            e = hy::launch_leaf_totals<float>((const float *)V.p->A, V.g, V.own, hole, nd, V.dv, V.partials, f->stream);
        std::vector<double> host((size_t)(V.rows * 5));
        if (e == hipSuccess)
            e = hipMemcpyAsync(host.data(), V.partials, sizeof(double) * host.size(), hipMemcpyDeviceToHost, f->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
        if (e != hipSuccess) return hip_fail(e, "leaf totals");
        for (int64_t r = 0; r < V.rows; ++r)
            for (int k = 0; k < 5; ++k) out[k] += host[(size_t)(r * 5 + k)];
    }
    return HY_OK;
}

hy_status hy_fmr_autotune(hy_fmr *f, int solver, int reps, hy_launch_cfg *best)
{
    if (!f) return fail(HY_EINVAL, "null handle");
    fmr_drop_graph(f);  // captured with the old launch shapes
    for (int l = 0; l < f->nlev; ++l) {
        hy_status st = hy_autotune(f->lev[l].p, solver, reps, best ? &best[l] : nullptr, nullptr);
        if (st != HY_OK) return st;
    }
    return HY_OK;
}

hy_status hy_fmr_destroy(hy_fmr *f)
{
    if (!f) return HY_OK;
    hipStreamSynchronize(f->stream);
    fmr_drop_graph(f);
    if (f->capture) (void)hipStreamDestroy(f->capture);
    for (int l = 0; l < f->nlev; ++l)
        if (f->lev[l].p) hy_destroy(f->lev[l].p);
    delete f;
    return HY_OK;
}

}  // extern "C"
