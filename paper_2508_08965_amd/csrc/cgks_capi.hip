// C ABI of the CGKS-5 library (declared in include/cgks.h).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cgks.h"
#include "cgks_device.h"

using namespace cgks;

namespace {
thread_local std::string g_err;

int fail(int code, const char *msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return CGKS_EHIP;
}

#define HIP_TRY(call, where)                          \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

constexpr int kMaxDtParts = 1024;
}  // namespace

struct cgks_ctx {
    int device = 0;
    std::vector<BlockView> blocks;
    long Ntot = 0;
    cgks_params user{};
    DevParams P{};
    Metrics M{};
    double *metric_mem = nullptr;
    DevConsts *K = nullptr;
    double *gp = nullptr;     // [3][2][4][20][Ntot]
    double *fo = nullptr;     // [3][4][30][Ntot]
    double *stash = nullptr;  // [80][Ntot]
    double *Kmf = nullptr;    // constant blocks of the matrix-core reconstruction
    int ngroups = 256;        // workgroups of the matrix-core reconstruction
    double *dt_part = nullptr;
    int nparts = 1;
    int *flag = nullptr;      // device error mask
    hipStream_t last = nullptr;
    bool stage1_done = false;
    // kernel timing
    bool prof = false;
    struct Pending { hipEvent_t a, b; int kind; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
};

namespace {
hipEvent_t get_event(cgks_ctx *c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// brackets one launch with events when profiling is on
struct Timed {
    cgks_ctx *c;
    hipStream_t s;
    int kind;
    hipEvent_t a = nullptr;
    Timed(cgks_ctx *c_, hipStream_t s_, int k) : c(c_), s(s_), kind(k) {
        if (c->prof) {
            a = get_event(c);
            (void)hipEventRecord(a, s);
        }
    }
    ~Timed() {
        if (c->prof) {
            hipEvent_t b = get_event(c);
            (void)hipEventRecord(b, s);
            c->pending.push_back({a, b, kind});
        }
    }
};
}  // namespace

static DevParams make_dev_params(const cgks_params &p) {
    DevParams d{};
    d.gamma = p.gamma;
    d.K = (5.0 - 3.0 * p.gamma) / (p.gamma - 1.0);
    d.cfl = p.cfl;
    d.tau_eps = p.tau_eps;
    d.tau_C = p.tau_C;
    d.mu0 = p.mu0;
    d.T_ref = p.T_ref;
    d.S_suth = p.S_suth;
    d.Pr = p.Pr;
    d.geno_C = p.geno_C;
    d.geno_eps = p.geno_eps;
    d.geno_r = p.geno_r;
    d.inv_tanhC = 1.0 / std::tanh(p.geno_C);
    d.viscous = p.viscous;
    d.visc_law = p.visc_law;
    d.tau_zero = p.tau_zero;
    d.linear = p.linear;
    d.prandtl_fix = p.prandtl_fix;
    return d;
}

static int check_params(const cgks_params *p) {
    if (!p) return fail(CGKS_EINVAL, "params is NULL");
    if (!(p->gamma > 1.0 && p->gamma < 5.0 / 3.0 + 1e-12)) return fail(CGKS_EINVAL, "gamma must be in (1, 5/3]");
    if (!(p->cfl > 0.0)) return fail(CGKS_EINVAL, "cfl must be positive");
    if (!(p->geno_C > 0.0) || !(p->geno_eps > 0.0) || !(p->geno_r > 0.0)) return fail(CGKS_EINVAL, "GENO constants must be positive");
    if (p->viscous && !(p->mu0 > 0.0)) return fail(CGKS_EINVAL, "viscous mode needs mu0 > 0");
    if (p->visc_law && (!(p->T_ref > 0.0) || !(p->S_suth >= 0.0))) return fail(CGKS_EINVAL, "Sutherland needs T_ref > 0, S >= 0");
    if (p->prandtl_fix && !(p->Pr > 0.0)) return fail(CGKS_EINVAL, "Pr must be positive");
    if (p->recon_prec < 0 || p->recon_prec > 2)
        return fail(CGKS_EUNSUPPORTED, "recon_prec must be 0 (FP64), 1 (FP32x3) or 2 (BF16x3)");
    if (p->flux_prec < 0 || p->flux_prec > 1) return fail(CGKS_EUNSUPPORTED, "flux_prec must be 0 (FP64) or 1 (FP32)");
    if (p->recon_impl != 0 && p->recon_impl != 1) return fail(CGKS_EINVAL, "recon_impl must be 0 or 1");
    if (p->recon_impl == 1 && (p->recon_prec != 0 || p->flux_prec != 0))
        return fail(CGKS_EUNSUPPORTED, "the vector-ALU reconstruction is FP64 only");
    return CGKS_OK;
}

// Gauss-point buffer in FP32 whenever the reconstruction or the flux runs in reduced precision;
// face buffer in FP32 when the flux does.  The state and the S2O4 accumulation stay FP64.
static bool gp32(const cgks_ctx *c) { return c->user.recon_prec != 0 || c->user.flux_prec != 0; }
static bool fo32(const cgks_ctx *c) { return c->user.flux_prec != 0; }

static hipError_t run_recon(cgks_ctx *ctx, const BlockView &b, const double *Q, const double *G, const double *L,
                            hipStream_t s) {
    if (ctx->user.recon_impl == 1) return launch_recon(b, ctx->Ntot, Q, G, L, ctx->M, ctx->K, ctx->P, ctx->gp, s);
    return launch_recon_mfma(ctx->user.recon_prec, gp32(ctx), b, ctx->Ntot, Q, G, L, ctx->M, ctx->Kmf, ctx->P, ctx->gp,
                             ctx->ngroups, s);
}

extern "C" {

void cgks_default_params(cgks_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->gamma = 1.4;
    p->cfl = 0.5;
    p->tau_eps = 0.05;
    p->tau_C = 5.0;
    p->mu0 = 0.0;
    p->T_ref = 1.0;
    p->S_suth = 0.0;
    p->Pr = 1.0;
    p->geno_C = 150.0;
    p->geno_eps = 1e-15;
    p->geno_r = 2.0;
}

const char *cgks_last_error(void) { return g_err.c_str(); }

long cgks_num_cells(const cgks_ctx *ctx) { return ctx ? ctx->Ntot : 0; }

void cgks_ctx_destroy(cgks_ctx *ctx) {
    if (!ctx) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->metric_mem);
    (void)hipFree(ctx->K);
    (void)hipFree(ctx->Kmf);
    (void)hipFree(ctx->gp);
    (void)hipFree(ctx->fo);
    (void)hipFree(ctx->stash);
    (void)hipFree(ctx->dt_part);
    (void)hipFree(ctx->flag);
    for (auto &p : ctx->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    (void)hipSetDevice(cur);
    delete ctx;
}

int cgks_ctx_create(cgks_ctx **out, int nblocks, const int *dims, const double *const *nodes, const cgks_params *p,
                    void *stream) {
    if (!out) return fail(CGKS_EINVAL, "out is NULL");
    *out = nullptr;
    if (nblocks < 1 || !dims || !nodes) return fail(CGKS_EINVAL, "need nblocks >= 1, dims and nodes");
    int st = check_params(p);
    if (st) return st;
    long Ntot = 0;
    std::vector<BlockView> blocks(nblocks);
    for (int b = 0; b < nblocks; ++b) {
        if (dims[3 * b] < 1 || dims[3 * b + 1] < 1 || dims[3 * b + 2] < 1) return fail(CGKS_EINVAL, "block dims must be >= 1");
        if (!nodes[b]) return fail(CGKS_EINVAL, "block nodes pointer is NULL");
        blocks[b].nx = dims[3 * b];
        blocks[b].ny = dims[3 * b + 1];
        blocks[b].nz = dims[3 * b + 2];
        blocks[b].N = (long)blocks[b].nx * blocks[b].ny * blocks[b].nz;
        blocks[b].off = Ntot;
        Ntot += blocks[b].N;
    }
    hipStream_t s = (hipStream_t)stream;
    cgks_ctx *c = new cgks_ctx();
    HIP_TRY(hipGetDevice(&c->device), "hipGetDevice");
    c->blocks = blocks;
    c->Ntot = Ntot;
    c->user = *p;
    c->P = make_dev_params(*p);
    auto alloc = [&](void **ptr, size_t bytes) -> bool { return hipMalloc(ptr, bytes) == hipSuccess; };
    const size_t nmet = 1 + 9 + 9 + 36 + 12 + 12;
    bool ok = alloc((void **)&c->metric_mem, sizeof(double) * nmet * Ntot) && alloc((void **)&c->K, sizeof(DevConsts)) &&
              alloc((void **)&c->Kmf, sizeof(double) * std::max(kMfmaBlocks * 64, kBfBlocks * 512)) &&
              alloc((void **)&c->gp, sizeof(double) * 480 * Ntot) && alloc((void **)&c->fo, sizeof(double) * 360 * Ntot) &&
              alloc((void **)&c->stash, sizeof(double) * 80 * Ntot) &&
              alloc((void **)&c->dt_part, sizeof(double) * kMaxDtParts) && alloc((void **)&c->flag, sizeof(int));
    if (!ok) {
        cgks_ctx_destroy(c);
        return fail(CGKS_ENOMEM, "device allocation failed");
    }
    double *mm = c->metric_mem;
    c->M.vol = mm;
    c->M.J0 = mm + Ntot;
    c->M.JiT = mm + 10 * Ntot;
    c->M.fn = mm + 19 * Ntot;
    c->M.fw = mm + 55 * Ntot;
    c->M.dtm = mm + 67 * Ntot;
    c->nparts = (int)std::min<long>(kMaxDtParts, (Ntot + 255) / 256);

    // constants of the standard cell
    HostConsts *hk = new HostConsts();
    build_constants(*hk);
    DevConsts dk;
    std::memcpy(dk.R, hk->R, sizeof dk.R);
    std::memcpy(dk.E, hk->E, sizeof dk.E);
    std::memcpy(dk.GL, hk->GL, sizeof dk.GL);
    std::memcpy(dk.GT, hk->GT, sizeof dk.GT);
    std::memcpy(dk.xg, hk->xg, sizeof dk.xg);
    std::vector<double> kmf(std::max(kMfmaBlocks * 64, kBfBlocks * 512));
    const bool packed = (p->recon_prec == 2) ? pack_mfma_bf16(*hk, kmf.data()) : pack_mfma(*hk, kmf.data(), p->recon_prec == 0);
    delete hk;
    if (!packed) {
        cgks_ctx_destroy(c);
        return fail(CGKS_EINVAL, "Gram matrices are not positive definite");
    }
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->ngroups = 2 * prop.multiProcessorCount;
    }
    int rc = CGKS_OK;
    do {
        hipError_t e = hipMemcpyAsync(c->K, &dk, sizeof dk, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(c->Kmf, kmf.data(), sizeof(double) * kmf.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { rc = hip_fail(e, "upload constants"); break; }
        e = hipMemsetAsync(c->flag, 0, sizeof(int), s);
        if (e != hipSuccess) { rc = hip_fail(e, "clear flag"); break; }
        for (int b = 0; b < nblocks && rc == CGKS_OK; ++b) {
            const BlockView &bv = c->blocks[b];
            size_t nn = (size_t)(bv.nx + 1) * (bv.ny + 1) * (bv.nz + 1) * 3;
            double *dn = nullptr;
            e = hipMalloc((void **)&dn, nn * sizeof(double));
            if (e != hipSuccess) { rc = hip_fail(e, "node buffer"); break; }
            e = hipMemcpyAsync(dn, nodes[b], nn * sizeof(double), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = launch_metrics(bv, dn, c->M, Ntot, c->flag, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            (void)hipFree(dn);
            if (e != hipSuccess) rc = hip_fail(e, "metrics");
        }
        if (rc) break;
        int bad = 0;
        e = hipMemcpy(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) { rc = hip_fail(e, "read flag"); break; }
        if (bad) { rc = fail(CGKS_EINVAL, "mesh has a cell with non-positive volume or det J0"); break; }
    } while (0);
    if (rc) {
        cgks_ctx_destroy(c);
        return rc;
    }
    c->last = s;
    *out = c;
    return CGKS_OK;
}

int cgks_dt(cgks_ctx *ctx, const double *Q, double *dt_dev, void *stream) {
    if (!ctx || !Q || !dt_dev) return fail(CGKS_EINVAL, "cgks_dt: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    Timed t(ctx, s, 0);
    HIP_TRY(launch_dt(0, ctx->Ntot, ctx->Ntot, Q, ctx->M.dtm, ctx->P, ctx->dt_part, ctx->nparts, ctx->flag, s), "dt");
    HIP_TRY(launch_dt_final(ctx->dt_part, ctx->nparts, dt_dev, s), "dt final");
    return CGKS_OK;
}

int cgks_stage(cgks_ctx *ctx, int stage, const double *dt_dev, double *Q, double *G, double *L, void *stream) {
    if (!ctx || !dt_dev || !Q || !G || !L) return fail(CGKS_EINVAL, "cgks_stage: NULL argument");
    if (stage != 1 && stage != 2) return fail(CGKS_EINVAL, "cgks_stage: stage must be 1 or 2");
    if (stage == 2 && !ctx->stage1_done) return fail(CGKS_EINVAL, "cgks_stage: stage 2 without a preceding stage 1");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    for (const BlockView &b : ctx->blocks) {
        {
            Timed t(ctx, s, 1);
            HIP_TRY(run_recon(ctx, b, Q, G, L, s), "recon");
        }
        {
            Timed t(ctx, s, 2);
            HIP_TRY(launch_flux(ctx->user.flux_prec, gp32(ctx), b, ctx->Ntot, ctx->gp, ctx->M, dt_dev, ctx->P, ctx->fo,
                                ctx->flag, s),
                    "flux");
        }
        {
            Timed t(ctx, s, 3);
            HIP_TRY(launch_update(stage, fo32(ctx), b, ctx->Ntot, ctx->fo, ctx->M, dt_dev, Q, G, L, ctx->stash, s),
                    "update");
        }
    }
    ctx->stage1_done = (stage == 1);
    return CGKS_OK;
}

int cgks_step(cgks_ctx *ctx, double *Q, double *G, double *L, double *dt_dev, int use_cfl, void *stream) {
    if (!ctx || !dt_dev || !Q || !G || !L) return fail(CGKS_EINVAL, "cgks_step: NULL argument");
    int st;
    if (use_cfl && (st = cgks_dt(ctx, Q, dt_dev, stream))) return st;
    if ((st = cgks_stage(ctx, 1, dt_dev, Q, G, L, stream))) return st;
    return cgks_stage(ctx, 2, dt_dev, Q, G, L, stream);
}

int cgks_check(cgks_ctx *ctx, int *flags_host) {
    if (!ctx || !flags_host) return fail(CGKS_EINVAL, "cgks_check: NULL argument");
    HIP_TRY(hipStreamSynchronize(ctx->last), "sync");
    int f = 0;
    HIP_TRY(hipMemcpy(&f, ctx->flag, sizeof(int), hipMemcpyDeviceToHost), "read flag");
    *flags_host = f;
    if (f) {
        HIP_TRY(hipMemset(ctx->flag, 0, sizeof(int)), "clear flag");
        return fail(CGKS_ENONPHYS, "non-physical state met by a kernel");
    }
    return CGKS_OK;
}

int cgks_recon(cgks_ctx *ctx, const double *Q, const double *G, const double *L, double *gp, void *stream) {
    if (!ctx || !Q || !G || !L || !gp) return fail(CGKS_EINVAL, "cgks_recon: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    for (const BlockView &b : ctx->blocks) {
        HIP_TRY(run_recon(ctx, b, Q, G, L, s), "recon");
        HIP_TRY(launch_gp_export(gp32(ctx), b, ctx->Ntot, ctx->gp, gp, s), "export");
    }
    return CGKS_OK;
}

int cgks_flux(cgks_ctx *ctx, long n, const double *ql, const double *gl, const double *qr, const double *gr,
              const double *nrm, const double *dt_dev, double *F, double *Ft, double *sides, void *stream) {
    if (!ctx || n < 0 || !ql || !gl || !qr || !gr || !nrm || !dt_dev || !F || !Ft || !sides)
        return fail(CGKS_EINVAL, "cgks_flux: bad argument");
    if (n == 0) return CGKS_OK;
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(launch_flux_points(ctx->user.flux_prec, n, ql, gl, qr, gr, nrm, dt_dev, ctx->P, F, Ft, sides, ctx->flag, s),
            "flux points");
    return CGKS_OK;
}

int cgks_metrics(cgks_ctx *ctx, double *vol, double *J0, double *fn, double *fw, void *stream) {
    if (!ctx) return fail(CGKS_EINVAL, "cgks_metrics: NULL context");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    const long N = ctx->Ntot;
    if (vol) HIP_TRY(hipMemcpyAsync(vol, ctx->M.vol, sizeof(double) * N, hipMemcpyDeviceToDevice, s), "copy vol");
    if (J0) HIP_TRY(hipMemcpyAsync(J0, ctx->M.J0, sizeof(double) * 9 * N, hipMemcpyDeviceToDevice, s), "copy J0");
    if (fn) HIP_TRY(hipMemcpyAsync(fn, ctx->M.fn, sizeof(double) * 36 * N, hipMemcpyDeviceToDevice, s), "copy fn");
    if (fw) HIP_TRY(hipMemcpyAsync(fw, ctx->M.fw, sizeof(double) * 12 * N, hipMemcpyDeviceToDevice, s), "copy fw");
    return CGKS_OK;
}

int cgks_profile(cgks_ctx *ctx, int enable) {
    if (!ctx) return fail(CGKS_EINVAL, "cgks_profile: NULL context");
    ctx->prof = enable != 0;
    return CGKS_OK;
}

int cgks_profile_read(cgks_ctx *ctx, double *ms, long *launches) {
    if (!ctx || !ms || !launches) return fail(CGKS_EINVAL, "cgks_profile_read: NULL argument");
    for (int k = 0; k < CGKS_NKINDS; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &p : ctx->pending) {
        HIP_TRY(hipEventSynchronize(p.b), "event sync");
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, p.a, p.b), "event time");
        ms[p.kind] += t;
        launches[p.kind] += 1;
        ctx->pool.push_back(p.a);
        ctx->pool.push_back(p.b);
    }
    ctx->pending.clear();
    return CGKS_OK;
}

}  // extern "C"
