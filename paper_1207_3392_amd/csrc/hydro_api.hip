// hydro_api.hip -- host runtime behind include/hydro.h: patch descriptors,
// workspace carving, stream-ordered launches, the device error latch and
// per-kernel event timing.
#include "hydro.h"
#include "hy_internal.h"
#include "hy_mlp.h"

#include <cmath>
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
    bool mlp_set = false;
    hipStream_t stream = nullptr;
    int parity = 0;
    hy::LaunchCfg cfg{64, 8, 32};
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev[2];
    int nrec[2] = {0, 0};
    double ms[2] = {0.0, 0.0};
    int64_t launches[2] = {0, 0};
};

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
    if (d->n[0] > (int64_t)1 << 20 || d->n[1] > (int64_t)1 << 20 || d->n[2] > (int64_t)1 << 20)
        return fail(HY_EINVAL, "dimension too large");
    const int64_t N = ncells(*d);
    // kernels address cells with 32-bit offsets within one variable's array
    const int64_t es = d->precision == 64 ? 8 : 4;
    if (N * es > ((int64_t)1 << 32) - 256)
        return fail(HY_EINVAL, "patch too large: one variable's array must stay below 4 GiB");
    return HY_OK;
}

struct Layout {
    size_t ctl, partials, A, B, slopes, mlp, total;
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
    L.A = o;
    o = align_up(o + es * nv * (size_t)L.vstride, 256);
    L.B = o;
    o = align_up(o + es * nv * (size_t)L.vstride, 256);
    L.slopes = o;
    if (d.limiter == HY_LIM_LEARNED) o = align_up(o + sizeof(float) * d.ndim * nv * (size_t)L.vstride, 256);
    L.total = o + 256;  // slack for aligning the caller's base pointer
    return L;
}

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
        a.n[q] = d.n[q];
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
    return a;
}

template <typename T>
hipError_t run_stage(hy_patch *p, int solver, int stage, int dt_mode, double dt, double cfl, double t_end)
{
    hipError_t e;
    if (p->d.limiter == HY_LIM_LEARNED) {
        const T *uin = (const T *)(stage == 1 ? p->A : p->B);
        e = hy::launch_learned_slopes((const float *)uin, p->slopes, p->d.n, p->vstride, p->d.ndim,
                                      (float)(p->d.gamma - 1.0), p->d.bc, p->mlp, p->stream);
        if (e != hipSuccess) return e;
    }
    const int k = stage - 1;
    const bool rec = p->timing && p->nrec[k] < kTimingPool;
    if (rec) {
        e = hipEventRecord(p->ev[k][2 * p->nrec[k]], p->stream);
        if (e != hipSuccess) return e;
    }
    hy::StageArgs<T> a = stage_args<T>(p, stage, dt_mode, dt, cfl, t_end);
    e = hy::launch_stage<T>(p->d.ndim, solver, stage, p->d.limiter, p->cfg, a, p->stream);
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

void pick_config(hy_patch *p)
{
    // plane tile and z chunk: a launch should have >= ~1024 workgroups
    const hy_patch_desc &d = p->d;
    p->cfg.bx = 64;
    p->cfg.by = d.ndim == 1 ? 1 : 8;
    if (d.ndim >= 2 && d.precision == 32) {
        p->cfg.bx = 32;
        p->cfg.by = 16;
    }
    if (const char *e = std::getenv("HY_TILE")) {  // "BXxBY", for tuning runs
        int bx = 0, by = 0;
        if (d.ndim > 1 && std::sscanf(e, "%dx%d", &bx, &by) == 2 &&
            ((bx == 64 && (by == 8 || by == 4)) || (bx == 32 && (by == 8 || (by == 16 && d.precision == 32))))) {
            p->cfg.bx = bx;
            p->cfg.by = by;
        }
    }
    if (d.ndim == 3) {
        const int64_t tiles = ((d.n[0] + p->cfg.bx - 1) / p->cfg.bx) * ((d.n[1] + p->cfg.by - 1) / p->cfg.by);
        int64_t chunks = (1024 + tiles - 1) / tiles;
        if (chunks > d.n[2] / 8) chunks = d.n[2] / 8;
        if (chunks < 1) chunks = 1;
        p->cfg.zchunk = (int)((d.n[2] + chunks - 1) / chunks);
    } else {
        p->cfg.zchunk = 1;
    }
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
    if (solver != HY_HLL && solver != HY_HLLC) return fail(HY_EINVAL, "unknown solver");
    if (p->d.limiter == HY_LIM_LEARNED && !p->mlp_set) return fail(HY_EINVAL, "learned limiter without weights");
    hipError_t e = one_step(p, solver, hy::DT_HOST, dt, 0.0, 0.0);
    if (e != hipSuccess) return hip_fail(e, "stage launch");
    return HY_OK;
}

hy_status hy_advance(hy_patch *p, int nsteps, double cfl, double t_end, int solver)
{
    if (!p) return fail(HY_EINVAL, "null patch");
    if (nsteps < 0) return fail(HY_EINVAL, "nsteps must be >= 0");
    if (!(cfl > 0.0) || !std::isfinite(cfl) || std::isnan(t_end)) return fail(HY_EINVAL, "bad cfl or t_end");
    if (solver != HY_HLL && solver != HY_HLLC) return fail(HY_EINVAL, "unknown solver");
    if (p->d.limiter == HY_LIM_LEARNED && !p->mlp_set) return fail(HY_EINVAL, "learned limiter without weights");
    for (int i = 0; i < nsteps; ++i) {
        hipError_t e = one_step(p, solver, hy::DT_DEVICE, 0.0, cfl, t_end);
        if (e != hipSuccess) return hip_fail(e, "stage launch");
    }
    return HY_OK;
}

hy_status hy_cfl_dt(hy_patch *p, double cfl, double *dt_out)
{
    if (!p || !dt_out) return fail(HY_EINVAL, "null argument");
    if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(HY_EINVAL, "cfl must be finite and > 0");
    hy::DevCtl c;
    hy_status st = read_ctl(p, &c);
    if (st != HY_OK) return st;
    const double rate = __builtin_bit_cast(double, c.rate[p->parity]);
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

hy_status hy_set_mlp(hy_patch *p, const float *w, size_t n)
{
    if (!p || !w) return fail(HY_EINVAL, "null argument");
    if (n != (size_t)hy::MLP_NPARAM) return fail(HY_EINVAL, "expected 1249 weights");
    hy::MlpDevice host;
    hy::mlp_pack(w, &host);
    hipError_t e = hipMemcpyAsync(p->mlp, &host, sizeof(host), hipMemcpyHostToDevice, p->stream);
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
    if (e != hipSuccess) return hip_fail(e, "synchronise");
    for (int k = 0; k < 2; ++k) {
        for (int i = 0; i < p->nrec[k]; ++i) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, p->ev[k][2 * i], p->ev[k][2 * i + 1]);
            if (e != hipSuccess) return hip_fail(e, "event elapsed");
            p->ms[k] += t;
        }
        p->launches[k] += p->nrec[k];
        p->nrec[k] = 0;
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

hy_status hy_destroy(hy_patch *p)
{
    if (!p) return HY_OK;
    hipStreamSynchronize(p->stream);
    for (int k = 0; k < 2; ++k)
        for (auto &ev : p->ev[k]) hipEventDestroy(ev);
    delete p;
    return HY_OK;
}

}  // extern "C"
