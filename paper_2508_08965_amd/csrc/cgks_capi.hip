// C ABI of the CGKS-5 library (declared in include/cgks.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cgks.h"
#include "cgks_device.h"
#include "cgks_mlp.h"

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

// Partial minima of cgks_dt_noalloc: a file-scope device array (one copy per GPU, held until
// the process ends) instead of context memory.  In host code its name is not a device address;
// each device's copy is looked up once, with that device current, by hipGetSymbolAddress, and
// only that pointer is used.
constexpr int kNoallocDtParts = 1024;  // 8 KB
static __device__ __align__(256) double scratch[kNoallocDtParts];

namespace {
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch;  // device -> address of its copy of `scratch`

// Address of `scratch` on the current device `dev` (looked up on the first call per device).
int scratch_address(int dev, double **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
        it = g_scratch.emplace(dev, (double *)p).first;
    }
    *out = it->second;
    return hipSuccess;
}
}  // namespace

struct cgks_ctx {
    int device = 0;
    std::vector<BlockView> blocks;
    std::vector<double *> dnodes;  // per block: its nodes on the device (diagnostics at Gauss points)
    long Ntot = 0;
    cgks_params user{};
    DevParams P{};
    Metrics M{};
    double *metric_mem = nullptr;
    DevConsts *K = nullptr;
    double *gp = nullptr;     // [3][2][4][20][Gtot] (padded rows: BlockView::gp_at)
    double *fo = nullptr;     // [3][4][30][Ntot]
    double *stash = nullptr;  // [80][Ntot]
    double *Kmf = nullptr;    // constant blocks of the matrix-core reconstruction
    double *pcm = nullptr;    // per-cell matrices (recon_impl 2), tiled by 64 cells
    double *dt_part = nullptr;
    double *dt_static = nullptr;  // this device's copy of `scratch` (cgks_dt_noalloc)
    double *diag_part = nullptr;  // [nparts][7] partial sums of the flow diagnostics
    void *wallf = nullptr;        // wall sides: F, F_t of the minus-side wall faces [4 kk][10][Wtot]
    long Wtot = 0;                // wall faces of the minus sides over every block and axis
    bool walls = false;
    int nparts = 1;
    int ncu = 256;
    // work lists of the reconstruction (1), flux (2) and update (3) kernels
    BlockView *d_blocks = nullptr;
    struct List {
        cgks_launch cfg{};
        std::vector<int> tile_cells;  // per block: run length, or brick x extent
        std::vector<int> by, bz;      // per block: brick extents in y and z (0: runs)
        std::vector<int> first;       // per block: index of its first tile; first[nblocks] = ntiles
        Tile *d = nullptr;
        int n = 0, cap = 0;
    } wl[4];
    // learned blend weights
    unsigned char *jump = nullptr;        // [Ntot] jump flags
    unsigned long long *jcount = nullptr; // flagged cells since the last read
    long long jexamined = 0;              // cells examined since the last read (host count)
    float *mlp_w = nullptr, *mlp_m = nullptr, *mlp_v = nullptr, *mlp_g = nullptr, *mlp_loss = nullptr;
    unsigned char *mlp_packed = nullptr;
    float *mlp_scratch = nullptr;
    long mlp_scratch_n = 0;
    int adam_t = 0;
    bool mlp_ready = false;
    // graph of one step
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void *gkey[4] = {nullptr, nullptr, nullptr, nullptr};
    int gkey_cfl = -1;
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
    d.weights = p.weights;
    d.jump_thresh = p.jump_thresh;
    for (int v = 0; v < 5; ++v) d.far[v] = p.farfield[v];
    d.inv_K3 = 1.0 / (d.K + 3.0);
    d.inv_Tref = (p.T_ref > 0.0) ? 1.0 / p.T_ref : 0.0;
    d.positivity = p.positivity;
    d.pos_eps = p.pos_eps;
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
    if (p->recon_impl < 0 || p->recon_impl > 2) return fail(CGKS_EINVAL, "recon_impl must be 0, 1 or 2");
    if (p->per_block != 0 && p->per_block != 1) return fail(CGKS_EINVAL, "per_block must be 0 or 1");
    if (p->positivity != 0 && p->positivity != 1) return fail(CGKS_EINVAL, "positivity must be 0 or 1");
    if (p->positivity && !(p->pos_eps > 0.0 && p->pos_eps < 1.0)) return fail(CGKS_EINVAL, "pos_eps must be in (0, 1)");
    if (p->weights != 0 && p->weights != 1) return fail(CGKS_EINVAL, "weights must be 0 (GENO) or 1 (learned)");
    if (!(p->jump_thresh >= 0.0)) return fail(CGKS_EINVAL, "jump_thresh must be >= 0");
    if (p->weights == 1 && (p->recon_impl != 0 || p->recon_prec != 0 || p->linear))
        return fail(CGKS_EUNSUPPORTED, "learned weights need the nonlinear FP64 matrix-core reconstruction");
    if (p->recon_impl != 0 && (p->recon_prec != 0 || p->flux_prec != 0))
        return fail(CGKS_EUNSUPPORTED, "the vector-ALU reconstruction is FP64 only");
    bool walls = false;
    for (int q = 0; q < 3; ++q) {
        const int a = p->bc[2 * q], b = p->bc[2 * q + 1];
        if (a < 0 || a > 4 || b < 0 || b > 4) return fail(CGKS_EINVAL, "bc entries must be 0, 1, 2, 3 or 4");
        if ((a == 0) != (b == 0)) return fail(CGKS_EINVAL, "the two sides of an axis are both periodic or both walls");
        walls = walls || a != 0;
    }
    if (walls && p->recon_impl != 0)
        return fail(CGKS_EUNSUPPORTED, "wall sides need the matrix-core reconstruction (recon_impl 0)");
    if (walls && p->positivity)
        return fail(CGKS_EUNSUPPORTED, "the interface-state limiter is for periodic blocks");
    for (int sd = 0; sd < 6; ++sd)
        if (p->bc[sd] == 4 && p->weights == 1)
            return fail(CGKS_EUNSUPPORTED, "learned weights are not available with non-reflecting sides");
    for (int sd = 0; sd < 6; ++sd)
        if (p->bc[sd] >= 3) {
            const double *f = p->farfield;
            const double ke = 0.5 * (f[1] * f[1] + f[2] * f[2] + f[3] * f[3]) / f[0];
            if (!(f[0] > 0.0) || !((p->gamma - 1.0) * (f[4] - ke) > 0.0))
                return fail(CGKS_EINVAL, "far-field state needs positive density and pressure");
        }
    return CGKS_OK;
}

// A wall side must be a plane normal to its axis, with the axis pointing into the block, and
// the tangential node coordinates of the two sides of the axis must agree: the wall faces of
// both sides then have the geometry of the plus side's face records (unit normal e_q).
static bool wall_geometry_ok(const double *nd, int nx, int ny, int nz, int q) {
    const int n[3] = {nx, ny, nz};
    auto at = [&](int i, int j, int k) {
        return nd + 3 * ((long)i + (long)(nx + 1) * ((long)j + (long)(ny + 1) * (long)k));
    };
    const int ta = (q == 0) ? 1 : 0, tb = (q == 2) ? 1 : 2;
    int idx[3] = {0, 0, 0};
    const double x0 = at(0, 0, 0)[q];
    idx[q] = n[q];
    const double x1 = at(idx[0], idx[1], idx[2])[q];
    double scale = 1.0;
    for (int r = 0; r < 3; ++r) scale = std::max(scale, std::fabs(at(idx[0], idx[1], idx[2])[r]));
    const double tol = 1e-12 * std::max(scale, std::fabs(x0));
    if (!(x1 > x0)) return false;
    for (int ib = 0; ib <= n[tb]; ++ib)
        for (int ia = 0; ia <= n[ta]; ++ia) {
            int lo[3], hi[3];
            lo[ta] = hi[ta] = ia;
            lo[tb] = hi[tb] = ib;
            lo[q] = 0;
            hi[q] = n[q];
            const double *pl = at(lo[0], lo[1], lo[2]), *ph = at(hi[0], hi[1], hi[2]);
            if (std::fabs(pl[q] - x0) > tol || std::fabs(ph[q] - x1) > tol) return false;
            if (std::fabs(pl[ta] - ph[ta]) > tol || std::fabs(pl[tb] - ph[tb]) > tol) return false;
        }
    return true;
}

// Gauss-point buffer in FP32 whenever the reconstruction or the flux runs in reduced precision;
// face buffer in FP32 when the flux does.  The state and the S2O4 accumulation stay FP64.
static bool gp32(const cgks_ctx *c) { return c->user.recon_prec != 0 || c->user.flux_prec != 0; }
static bool fo32(const cgks_ctx *c) { return c->user.flux_prec != 0; }

// Work list of kernel kind k restricted to block b (b < 0: every block).
static WorkList work_list(const cgks_ctx *c, int k, int b) {
    const cgks_ctx::List &l = c->wl[k];
    WorkList w{c->d_blocks, l.d, l.n, l.cfg.xcd};
    if (b >= 0) {
        w.tiles = l.d + l.first[b];
        w.ntiles = l.first[b + 1] - l.first[b];
    }
    return w;
}

// Tiles of every block for kind k with the per-block tile sizes of the list, uploaded to the
// device (synchronous).
static hipError_t build_list(cgks_ctx *c, int k) {
    cgks_ctx::List &l = c->wl[k];
    std::vector<Tile> t;
    const int nb = (int)c->blocks.size();
    l.first.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        l.first[b] = (int)t.size();
        const BlockView &bv = c->blocks[b];
        const long T = l.tile_cells[b];
        const int by = l.by.empty() ? 0 : l.by[b], bz = l.bz.empty() ? 0 : l.bz[b];
        if (by > 0) {
            // the fewest bricks of at most by x bz rows that cover the block, with extents in y
            // and z that differ by at most one (no thin remainder brick whose rows would leave
            // most waves of the workgroup idle)
            const int ny_b = (bv.ny + by - 1) / by, nz_b = (bv.nz + bz - 1) / bz;
            for (int kz = 0, z0 = 0; kz < nz_b; ++kz) {
                const int ez = bv.nz / nz_b + (kz < bv.nz % nz_b ? 1 : 0);
                for (int ky = 0, y0 = 0; ky < ny_b; ++ky) {
                    const int ey = bv.ny / ny_b + (ky < bv.ny % ny_b ? 1 : 0);
                    for (int x0 = 0; x0 < bv.nx; x0 += (int)T)
                        t.push_back(Tile{b, (int)std::min<long>(T, bv.nx - x0),
                                         x0 + (long)bv.nx * (y0 + (long)bv.ny * z0), ey, ez, 0, 0});
                    y0 += ey;
                }
                z0 += ez;
            }
        } else {
            // a short first run up to the next multiple of 16 cells of the whole mesh, so that
            // every later chunk of 16 cells, a wave's row, starts on a 128-byte boundary of the
            // component arrays (a chunk across two cache lines costs its stores a second line)
            const long a = std::min<long>((16 - bv.off % 16) % 16, bv.N);
            if (a > 0) t.push_back(Tile{b, (int)a, 0, 0, 0, 0, 0});
            for (long st = a; st < bv.N; st += T) t.push_back(Tile{b, (int)std::min(T, bv.N - st), st, 0, 0, 0, 0});
        }
    }
    l.first[nb] = (int)t.size();
    if ((int)t.size() > l.cap) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        (void)hipFree(l.d);
        l.d = nullptr;
        l.cap = 0;
        e = hipMalloc((void **)&l.d, sizeof(Tile) * t.size());
        if (e != hipSuccess) return e;
        l.cap = (int)t.size();
    }
    l.n = (int)t.size();
    return hipMemcpy(l.d, t.data(), sizeof(Tile) * t.size(), hipMemcpyHostToDevice);
}

static void drop_graph(cgks_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->gkey_cfl = -1;
}

static hipError_t run_recon(cgks_ctx *ctx, int b, const double *Q, const double *G, const double *L, hipStream_t s) {
    if (ctx->user.recon_impl != 0) {
        // vector-ALU reference kernel (1) or per-cell stored matrices (2): one launch per block
        for (int i = 0; i < (int)ctx->blocks.size(); ++i) {
            if (b >= 0 && i != b) continue;
            hipError_t e = (ctx->user.recon_impl == 1)
                               ? launch_recon(ctx->blocks[i], ctx->Ntot, Q, G, L, ctx->M, ctx->K, ctx->P, ctx->gp, s)
                               : launch_recon_percell(ctx->blocks[i], ctx->Ntot, Q, G, L, ctx->M, ctx->K, ctx->P,
                                                      ctx->pcm, ctx->gp, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    BlendIO io{ctx->jump, ctx->mlp_packed, nullptr, nullptr};
    if (ctx->P.weights == 1) {
        hipError_t e = launch_jump(work_list(ctx, 3, b), ctx->Ntot, Q, ctx->P, ctx->jump, ctx->jcount, s);
        if (e != hipSuccess) return e;
        ctx->jexamined += (b < 0) ? ctx->Ntot : ctx->blocks[b].N;
    }
    return launch_recon_mfma(ctx->user.recon_prec, gp32(ctx), work_list(ctx, 1, b), ctx->Ntot, Q, G, L, ctx->M,
                             ctx->Kmf, ctx->P, ctx->gp, ctx->wl[1].cfg.ngroups, io, false, ctx->wl[1].cfg.stage != 0,
                             s);
}

// Q: the stage's cell averages (read only by the interface-state limiter, positivity = 1)
static hipError_t run_flux(cgks_ctx *ctx, int b, const double *dt_dev, const double *Q, hipStream_t s,
                           bool full = true) {
    hipError_t e = launch_flux(ctx->user.flux_prec, gp32(ctx), work_list(ctx, 2, b), ctx->Ntot, ctx->gp, ctx->M,
                               dt_dev, ctx->P, ctx->fo, ctx->flag, full, Q, s);
    // wall faces: recomputed against the mirrored interior state after the periodic pass
    for (int i = 0; i < (int)ctx->blocks.size() && e == hipSuccess && ctx->walls; ++i) {
        if (b >= 0 && i != b) continue;
        for (int q = 0; q < 3 && e == hipSuccess; ++q)
            if ((ctx->blocks[i].wall >> (2 * q)) & 1)
                e = launch_flux_wall(ctx->user.flux_prec, gp32(ctx), ctx->blocks[i], q, ctx->Ntot, ctx->gp, ctx->M,
                                     dt_dev, ctx->P, ctx->fo, ctx->wallf, ctx->Wtot, ctx->flag, full, s);
    }
    return e;
}

static hipError_t run_update(cgks_ctx *ctx, int stage, int b, const double *dt_dev, double *Q, double *G, double *L,
                             hipStream_t s) {
    return launch_update(stage, fo32(ctx), work_list(ctx, 3, b), ctx->Ntot, ctx->fo, ctx->M, dt_dev, Q, G, L,
                         ctx->stash, ctx->wl[3].cfg.ngroups, ctx->walls ? ctx->wallf : nullptr, ctx->Wtot, s);
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
    p->jump_thresh = 0.05;
    p->positivity = 0;
    p->pos_eps = 1e-3;
}

const char *cgks_last_error(void) { return g_err.c_str(); }

long cgks_num_cells(const cgks_ctx *ctx) { return ctx ? ctx->Ntot : 0; }

void cgks_ctx_destroy(cgks_ctx *ctx) {
    if (!ctx) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (double *dn : ctx->dnodes) (void)hipFree(dn);
    (void)hipFree(ctx->metric_mem);
    (void)hipFree(ctx->K);
    (void)hipFree(ctx->Kmf);
    (void)hipFree(ctx->pcm);
    (void)hipFree(ctx->wallf);
    (void)hipFree(ctx->diag_part);
    (void)hipFree(ctx->gp);
    (void)hipFree(ctx->fo);
    (void)hipFree(ctx->stash);
    (void)hipFree(ctx->dt_part);
    (void)hipFree(ctx->flag);
    (void)hipFree(ctx->d_blocks);
    (void)hipFree(ctx->jump);
    (void)hipFree(ctx->jcount);
    (void)hipFree(ctx->mlp_w);
    (void)hipFree(ctx->mlp_m);
    (void)hipFree(ctx->mlp_v);
    (void)hipFree(ctx->mlp_g);
    (void)hipFree(ctx->mlp_loss);
    (void)hipFree(ctx->mlp_packed);
    (void)hipFree(ctx->mlp_scratch);
    for (auto &l : ctx->wl) (void)hipFree(l.d);
    drop_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
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
        if (Ntot >= kMaxCells) return fail(CGKS_EINVAL, "total number of cells must be below 2^27");
    }
    // Gauss-point buffer: rows padded to a multiple of 16 cells where that costs at most a
    // quarter more (a block a few cells wide keeps its rows), block starts on 16 cells
    long Gtot = 0;
    for (BlockView &bv : blocks) {
        const int nxp = 16 * ((bv.nx + 15) / 16);
        bv.nxp = (4 * nxp <= 5 * bv.nx) ? nxp : bv.nx;
        bv.goff = Gtot;
        Gtot += 16 * (((long)bv.nxp * bv.ny * bv.nz + 15) / 16);
    }
    for (BlockView &bv : blocks) bv.gstride = Gtot;
    // wall sides (the same for every block): geometry check on the host nodes, wall-face offsets
    long Wtot = 0;
    for (int b = 0; b < nblocks; ++b) {
        BlockView &bv = blocks[b];
        bv.wall = 0;
        for (int q = 0; q < 3; ++q) {
            bv.wbase[q] = -1;
            if (!p->bc[2 * q]) continue;
            if (!wall_geometry_ok(nodes[b], bv.nx, bv.ny, bv.nz, q))
                return fail(CGKS_EINVAL, "a wall side is not a plane normal to its axis, or the two sides of the axis "
                                         "do not share their tangential node coordinates");
            for (int sd = 0; sd < 2; ++sd) {
                bv.wall |= 1 << (2 * q + sd);
                if (p->bc[2 * q + sd] == 2) bv.wall |= 1 << (8 + 2 * q + sd);
                if (p->bc[2 * q + sd] == 3) bv.wall |= 1 << (16 + 2 * q + sd);
                if (p->bc[2 * q + sd] == 4) bv.wall |= 1 << (24 + 2 * q + sd);
            }
            bv.wbase[q] = Wtot;
            Wtot += bv.N / ((q == 0) ? bv.nx : (q == 1) ? bv.ny : bv.nz);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    cgks_ctx *c = new cgks_ctx();
    HIP_TRY(hipGetDevice(&c->device), "hipGetDevice");
    {
        const int e = scratch_address(c->device, &c->dt_static);
        if (e != hipSuccess) {
            delete c;
            return hip_fail((hipError_t)e, "hipGetSymbolAddress(scratch)");
        }
    }
    c->blocks = blocks;
    c->Ntot = Ntot;
    c->Wtot = Wtot;
    c->walls = Wtot > 0;
    c->user = *p;
    c->P = make_dev_params(*p);
    auto alloc = [&](void **ptr, size_t bytes) -> bool { return hipMalloc(ptr, bytes) == hipSuccess; };
    const size_t nmet = 1 + 9 + 9 + 36 + 12 + 12;
    bool ok = alloc((void **)&c->metric_mem, sizeof(double) * nmet * Ntot) && alloc((void **)&c->K, sizeof(DevConsts)) &&
              alloc((void **)&c->Kmf, sizeof(double) * std::max(kMfmaBlocks * 64, kBfBlocks * 512)) &&
              alloc((void **)&c->gp, sizeof(double) * 480 * Gtot) && alloc((void **)&c->fo, sizeof(double) * 360 * Ntot) &&
              alloc((void **)&c->stash, sizeof(double) * 80 * Ntot) &&
              alloc((void **)&c->dt_part, sizeof(double) * kMaxDtParts) && alloc((void **)&c->flag, sizeof(int)) &&
              alloc((void **)&c->diag_part, sizeof(double) * 7 * kMaxDtParts) &&
              alloc((void **)&c->jump, Ntot) && alloc((void **)&c->jcount, sizeof(unsigned long long)) &&
              alloc((void **)&c->mlp_w, sizeof(float) * kMlpParams) &&
              alloc((void **)&c->mlp_m, sizeof(float) * kMlpParams) &&
              alloc((void **)&c->mlp_v, sizeof(float) * kMlpParams) &&
              alloc((void **)&c->mlp_g, sizeof(float) * kMlpParams) && alloc((void **)&c->mlp_loss, sizeof(float)) &&
              alloc((void **)&c->mlp_packed, kMlpPackBytes) &&
              (Wtot == 0 || alloc(&c->wallf, sizeof(double) * 40 * Wtot)) &&
              (p->recon_impl != 2 ||
               alloc((void **)&c->pcm, sizeof(double) * kPcElems *
                                           ((Ntot + kPcTile - 1) / kPcTile * kPcTile)));
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
    std::memcpy(dk.V, hk->V, sizeof dk.V);
    std::memcpy(dk.xv, hk->xv, sizeof dk.xv);
    std::memcpy(dk.wv, hk->wv, sizeof dk.wv);
    std::vector<double> kmf(std::max(kMfmaBlocks * 64, kBfBlocks * 512));
    const bool packed = (p->recon_prec == 2) ? pack_mfma_bf16(*hk, kmf.data()) : pack_mfma(*hk, kmf.data(), p->recon_prec == 0);
    delete hk;
    if (!packed) {
        cgks_ctx_destroy(c);
        return fail(CGKS_EINVAL, "Gram matrices are not positive definite");
    }
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->ncu = prop.multiProcessorCount;
    }
    // reconstruction: bricks staged in LDS (FP64 and FP32x3), else runs of 1536 cells (fewer
    // workgroups stage the constants)
    c->wl[1].cfg = (p->recon_prec != 2 && p->recon_impl == 0)
                       ? cgks_launch{kStgTile[0], 0, 0, kStgTile[1], kStgTile[2], 1}
                       : cgks_launch{1536, 0, 0, 0, 0, 0};
    c->wl[2].cfg = cgks_launch{kFluxTile, 0, 0, 0, 0, 0};
    c->wl[3].cfg = cgks_launch{kUpdateTile, 0, 0, 0, 0, 0};
    int rc = CGKS_OK;
    do {
        hipError_t e = hipMemcpyAsync(c->K, &dk, sizeof dk, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(c->Kmf, kmf.data(), sizeof(double) * kmf.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { rc = hip_fail(e, "upload constants"); break; }
        e = hipMemsetAsync(c->flag, 0, sizeof(int), s);
        if (e == hipSuccess) e = hipMemsetAsync(c->jcount, 0, sizeof(unsigned long long), s);
        if (e == hipSuccess) e = hipMemsetAsync(c->jump, 0, Ntot, s);
        if (e != hipSuccess) { rc = hip_fail(e, "clear flags"); break; }
        for (int b = 0; b < nblocks && rc == CGKS_OK; ++b) {
            const BlockView &bv = c->blocks[b];
            size_t nn = (size_t)(bv.nx + 1) * (bv.ny + 1) * (bv.nz + 1) * 3;
            double *dn = nullptr;
            e = hipMalloc((void **)&dn, nn * sizeof(double));
            if (e != hipSuccess) { rc = hip_fail(e, "node buffer"); break; }
            c->dnodes.push_back(dn);  // kept: the diagnostics integrate over each cell's trilinear map
            e = hipMemcpyAsync(dn, nodes[b], nn * sizeof(double), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = launch_metrics(bv, dn, c->M, Ntot, c->flag, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) rc = hip_fail(e, "metrics");
        }
        if (rc) break;
        int bad = 0;
        e = hipMemcpy(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) { rc = hip_fail(e, "read flag"); break; }
        if (bad) { rc = fail(CGKS_EINVAL, "mesh has a cell with non-positive volume or det J0"); break; }
        if (c->pcm) {
            for (int b = 0; b < nblocks && e == hipSuccess; ++b)
                e = launch_percell_setup(c->blocks[b], Ntot, c->M, c->K, c->pcm, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { rc = hip_fail(e, "per-cell matrices"); break; }
        }
        e = hipMalloc((void **)&c->d_blocks, sizeof(BlockView) * nblocks);
        if (e == hipSuccess)
            e = hipMemcpy(c->d_blocks, c->blocks.data(), sizeof(BlockView) * nblocks, hipMemcpyHostToDevice);
        for (int k = 1; k <= 3 && e == hipSuccess; ++k) {
            c->wl[k].tile_cells.assign(nblocks, c->wl[k].cfg.tile_cells);
            c->wl[k].by.assign(nblocks, c->wl[k].cfg.brick_y);
            c->wl[k].bz.assign(nblocks, c->wl[k].cfg.brick_z);
            e = build_list(c, k);
        }
        if (e != hipSuccess) { rc = hip_fail(e, "work lists"); break; }
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

int cgks_dt_noalloc(cgks_ctx *ctx, const double *Q, double *dt_dev, void *stream) {
    if (!ctx || !Q || !dt_dev) return fail(CGKS_EINVAL, "cgks_dt_noalloc: NULL argument");
    if (ctx->nparts > kNoallocDtParts)
        return fail(CGKS_EINVAL, "cgks_dt_noalloc: partition larger than the static scratch (1024 partial minima)");
    if (!ctx->dt_static) return fail(CGKS_EHIP, "cgks_dt_noalloc: no static scratch on this device");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(launch_dt(0, ctx->Ntot, ctx->Ntot, Q, ctx->M.dtm, ctx->P, ctx->dt_static, ctx->nparts, ctx->flag, s),
            "dt (static scratch)");
    HIP_TRY(launch_dt_final(ctx->dt_static, ctx->nparts, dt_dev, s), "dt final (static scratch)");
    return CGKS_OK;
}

int cgks_diagnostics(cgks_ctx *ctx, const double *Q, const double *G, double *out, void *stream) {
    if (!ctx || !Q || !G || !out) return fail(CGKS_EINVAL, "cgks_diagnostics: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(launch_diagnostics(ctx->Ntot, Q, G, ctx->M.vol, ctx->P, ctx->diag_part, ctx->nparts, out, s),
            "diagnostics");
    return CGKS_OK;
}

int cgks_diagnostics_hq(cgks_ctx *ctx, const double *Q, const double *G, const double *L, double *out,
                        void *stream) {
    if (!ctx || !Q || !G || !L || !out) return fail(CGKS_EINVAL, "cgks_diagnostics_hq: NULL argument");
    if (ctx->walls) return fail(CGKS_EUNSUPPORTED, "cgks_diagnostics_hq: periodic blocks only");
    const int nb = (int)ctx->blocks.size();
    if (nb > kMaxDtParts) return fail(CGKS_EUNSUPPORTED, "cgks_diagnostics_hq: at most 1024 blocks");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    // each block's cells in a fixed number of parts: deterministic sums; the coefficients go
    // to the Gauss-point buffer (a stage rebuilds it; stage 2 reads only the stash)
    const int per = kMaxDtParts / nb;
    int at = 0;
    for (int b = 0; b < nb; ++b) {
        const BlockView &bv = ctx->blocks[b];
        const int np = (int)std::max<long>(1, std::min<long>(per, (bv.N + 255) / 256));
        HIP_TRY(launch_diagnostics_hq(bv, ctx->Ntot, Q, G, L, ctx->dnodes[b], ctx->M, ctx->K, ctx->P, ctx->gp,
                                      ctx->diag_part + 7L * at, np, s),
                "diagnostics (Gauss points)");
        at += np;
    }
    HIP_TRY(launch_diagnostics_final(ctx->diag_part, at, out, s), "diagnostics final");
    return CGKS_OK;
}

int cgks_qcriterion(cgks_ctx *ctx, const double *Q, const double *G, double *out, void *stream) {
    if (!ctx || !Q || !G || !out) return fail(CGKS_EINVAL, "cgks_qcriterion: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(launch_qcriterion(ctx->Ntot, Q, G, out, s), "qcriterion");
    return CGKS_OK;
}

int cgks_stage(cgks_ctx *ctx, int stage, const double *dt_dev, double *Q, double *G, double *L, void *stream) {
    if (!ctx || !dt_dev || !Q || !G || !L) return fail(CGKS_EINVAL, "cgks_stage: NULL argument");
    if (stage != 1 && stage != 2) return fail(CGKS_EINVAL, "cgks_stage: stage must be 1 or 2");
    if (stage == 2 && !ctx->stage1_done) return fail(CGKS_EINVAL, "cgks_stage: stage 2 without a preceding stage 1");
    if (ctx->P.weights == 1 && !ctx->mlp_ready) return fail(CGKS_EINVAL, "learned weights: no MLP parameters set");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    const int nb = ctx->user.per_block ? (int)ctx->blocks.size() : 1;
    for (int i = 0; i < nb; ++i) {
        const int b = ctx->user.per_block ? i : -1;
        {
            Timed t(ctx, s, 1);
            HIP_TRY(run_recon(ctx, b, Q, G, L, s), "recon");
        }
        {
            Timed t(ctx, s, stage == 1 ? 2 : 4);
            HIP_TRY(run_flux(ctx, b, dt_dev, Q, s, stage == 1), "flux");
        }
        {
            Timed t(ctx, s, stage == 1 ? 3 : 5);
            HIP_TRY(run_update(ctx, stage, b, dt_dev, Q, G, L, s), "update");
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
    if (ctx->P.weights == 1 && !ctx->mlp_ready) return fail(CGKS_EINVAL, "learned weights: no MLP parameters set");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(run_recon(ctx, -1, Q, G, L, s), "recon");
    for (const BlockView &b : ctx->blocks) HIP_TRY(launch_gp_export(gp32(ctx), b, ctx->Ntot, ctx->gp, gp, s), "export");
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

int cgks_get_launch(const cgks_ctx *ctx, int kind, cgks_launch *out) {
    if (!ctx || !out) return fail(CGKS_EINVAL, "cgks_get_launch: NULL argument");
    if (kind < 1 || kind > 3) return fail(CGKS_EINVAL, "cgks_get_launch: kind must be 1, 2 or 3");
    *out = ctx->wl[kind].cfg;
    return CGKS_OK;
}

static int check_launch(const cgks_ctx *ctx, int kind, const cgks_launch &c) {
    if (kind < 1 || kind > 3) return fail(CGKS_EINVAL, "launch kind must be 1, 2 or 3");
    if (kind == 1 && (c.tile_cells < 16 || c.tile_cells > 4096 || c.tile_cells % 16))
        return fail(CGKS_EINVAL, "reconstruction tiles must be a multiple of 16 cells in [16, 4096]");
    if (c.brick_y < 0 || c.brick_z < 0 || (c.brick_y > 0) != (c.brick_z > 0) || c.brick_y > 4096 || c.brick_z > 4096)
        return fail(CGKS_EINVAL, "brick_y and brick_z must both be 0 (runs) or both in [1, 4096]");
    if (kind != 1 && c.brick_y != 0) return fail(CGKS_EINVAL, "bricks are for the reconstruction only");
    if (c.stage != 0 && c.stage != 1) return fail(CGKS_EINVAL, "stage must be 0 or 1");
    if (c.stage && (kind != 1 || c.tile_cells != 16 || c.brick_y < 1 ||
                    kStgRow * (c.brick_y + 2) * (c.brick_z + 2) > kStgCells))
        return fail(CGKS_EINVAL, "staged reconstruction: bricks of 16 x brick_y x brick_z cells with "
                                 "(brick_y + 2)(brick_z + 2) <= 120");
    if (c.stage && (ctx->user.recon_prec == 2 || ctx->user.recon_impl != 0))
        return fail(CGKS_EUNSUPPORTED, "staged reconstruction: FP64 or FP32x3 matrix-core reconstruction only");
    if (kind == 2 && (c.tile_cells != kFluxTile || c.ngroups != 0))
        return fail(CGKS_EINVAL, "flux: tiles of 128 cells, one workgroup per unit (ngroups 0)");
    if (kind == 3 && c.tile_cells != kUpdateTile) return fail(CGKS_EINVAL, "update tiles are 256 cells");
    if (c.ngroups < 0 || c.ngroups > 64 * ctx->ncu) return fail(CGKS_EINVAL, "ngroups must be in [0, 64 x CUs]");
    if (c.xcd != 0 && c.xcd != 1) return fail(CGKS_EINVAL, "xcd must be 0 or 1");
    if (c.xcd && kind != 2 && c.ngroups % 8) return fail(CGKS_EINVAL, "XCD order needs ngroups a multiple of 8");
    return CGKS_OK;
}

int cgks_set_launch(cgks_ctx *ctx, int kind, const cgks_launch *cfg) {
    if (!ctx || !cfg) return fail(CGKS_EINVAL, "cgks_set_launch: NULL argument");
    int st = check_launch(ctx, kind, *cfg);
    if (st) return st;
    HIP_TRY(hipDeviceSynchronize(), "sync");
    drop_graph(ctx);
    ctx->wl[kind].cfg = *cfg;
    ctx->wl[kind].tile_cells.assign(ctx->blocks.size(), cfg->tile_cells);
    ctx->wl[kind].by.assign(ctx->blocks.size(), cfg->brick_y);
    ctx->wl[kind].bz.assign(ctx->blocks.size(), cfg->brick_z);
    HIP_TRY(build_list(ctx, kind), "work list");
    return CGKS_OK;
}

int cgks_autotune(cgks_ctx *ctx, const double *Q, const double *G, const double *L, const double *dt_dev, int reps,
                  double *report, int report_len, void *stream) {
    if (!ctx || !Q || !G || !L || !dt_dev) return fail(CGKS_EINVAL, "cgks_autotune: NULL argument");
    if (reps < 1) return fail(CGKS_EINVAL, "cgks_autotune: reps must be >= 1");
    if (report && report_len < 1) return fail(CGKS_EINVAL, "cgks_autotune: report_len must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(hipDeviceSynchronize(), "sync");
    drop_graph(ctx);
    hipEvent_t e0 = get_event(ctx), e1 = get_event(ctx);
    int nrep = 0;
    auto note = [&](int kind, const cgks_launch &c, double ms) {
        if (!report) return;
        const int at = 1 + 7 * nrep;
        if (at + 7 > report_len) return;
        report[at] = kind;
        report[at + 1] = c.tile_cells;
        report[at + 2] = c.ngroups;
        report[at + 3] = c.xcd;
        report[at + 4] = c.brick_y;
        report[at + 5] = c.brick_z;
        report[at + 6] = ms;
        report[0] = ++nrep;
    };
    // mean milliseconds of `reps` launches after one untimed launch
    auto timeit = [&](auto &&launch, double &ms) -> hipError_t {
        hipError_t e = launch();
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        ms = (double)t / reps;
        return e;
    };
    const bool saved_prof = ctx->prof;
    ctx->prof = false;
    int rc = CGKS_OK;
    const int nb = (int)ctx->blocks.size();
    do {
        hipError_t e = hipSuccess;
        if (ctx->user.recon_impl == 0) {
            // 1) reconstruction tile size per block-size class, on a list of that class's blocks
            cgks_ctx::List &l = ctx->wl[1];
            const long lim[2] = {1L << 17, 1L << 19};
            auto cls = [&](long N) { return N < lim[0] ? 0 : (N < lim[1] ? 1 : 2); };
            // candidates: runs of 64..2048 cells and bricks (x, y, z extents) that march along z
            const int ncand = 12;
            const int cand[ncand][3] = {{64, 0, 0},   {128, 0, 0},  {256, 0, 0}, {512, 0, 0},
                                        {1024, 0, 0}, {1536, 0, 0}, {2048, 0, 0}, {16, 8, 16},
                                        {16, 8, 64},  {32, 4, 32},  {16, 16, 16}, {64, 2, 32}};
            const cgks_launch base = l.cfg;
            std::vector<int> best_c(3, -1);
            for (int k = 0; k < 3 && e == hipSuccess; ++k) {
                bool any = false;
                for (int b = 0; b < nb; ++b) any |= cls(ctx->blocks[b].N) == k;
                if (!any) continue;
                double bestms = 1e300;
                for (int ci = 0; ci < ncand && e == hipSuccess; ++ci) {
                    for (int b = 0; b < nb; ++b) {
                        l.tile_cells[b] = cand[ci][0];
                        l.by[b] = cand[ci][1];
                        l.bz[b] = cand[ci][2];
                    }
                    e = build_list(ctx, 1);
                    if (e != hipSuccess) break;
                    // blocks of a class are not contiguous: time each block's sub-list and sum
                    double ms_sum = 0.0;
                    for (int b = 0; b < nb && e == hipSuccess; ++b) {
                        if (cls(ctx->blocks[b].N) != k) continue;
                        const WorkList w = work_list(ctx, 1, b);
                        double ms = 0.0;
                        e = timeit([&] { return launch_recon_mfma(ctx->user.recon_prec, gp32(ctx), w, ctx->Ntot, Q, G, L,
                                                                  ctx->M, ctx->Kmf, ctx->P, ctx->gp, base.ngroups,
                                                                  BlendIO{ctx->jump, ctx->mlp_packed, nullptr, nullptr},
                                                                  false, false, s); },
                                   ms);
                        ms_sum += ms;
                    }
                    if (e != hipSuccess) break;
                    note(1, cgks_launch{cand[ci][0], base.ngroups, base.xcd, cand[ci][1], cand[ci][2], 0}, ms_sum);
                    if (ms_sum < bestms) {
                        bestms = ms_sum;
                        best_c[k] = ci;
                    }
                }
            }
            if (e != hipSuccess) break;
            for (int b = 0; b < nb; ++b) {
                const int ci = best_c[cls(ctx->blocks[b].N)];
                l.tile_cells[b] = ci >= 0 ? cand[ci][0] : base.tile_cells;
                l.by[b] = ci >= 0 ? cand[ci][1] : base.brick_y;
                l.bz[b] = ci >= 0 ? cand[ci][2] : base.brick_z;
            }
            e = build_list(ctx, 1);
            if (e != hipSuccess) break;
            l.cfg.tile_cells = l.tile_cells[0];
            l.cfg.brick_y = l.by[0];
            l.cfg.brick_z = l.bz[0];
            l.cfg.stage = 0;  // these candidates gather from memory; the staged form is timed below
            // 2) grid and XCD order over the whole list
            const int grids[4] = {ctx->ncu, 2 * ctx->ncu, 4 * ctx->ncu, 0};
            double best = 1e300;
            cgks_launch pick = l.cfg;
            for (int gi = 0; gi < 4 && e == hipSuccess; ++gi)
                for (int x = 0; x < 2 && e == hipSuccess; ++x) {
                    if (x && grids[gi] % 8) continue;
                    l.cfg.ngroups = grids[gi];
                    l.cfg.xcd = x;
                    const WorkList w = work_list(ctx, 1, -1);
                    double ms = 0.0;
                    e = timeit([&] { return launch_recon_mfma(ctx->user.recon_prec, gp32(ctx), w, ctx->Ntot, Q, G, L,
                                                              ctx->M, ctx->Kmf, ctx->P, ctx->gp, grids[gi],
                                                              BlendIO{ctx->jump, ctx->mlp_packed, nullptr, nullptr},
                                                              false, false, s); },
                               ms);
                    note(1, l.cfg, ms);
                    if (ms < best) {
                        best = ms;
                        pick = l.cfg;
                    }
                }
            l.cfg.ngroups = pick.ngroups;
            l.cfg.xcd = pick.xcd;
            if (e != hipSuccess) break;
            // 2b) the bricks staged in LDS (one form for the whole list), against the pick
            if (ctx->user.recon_prec != 2) {
                const std::vector<int> tc = l.tile_cells, by = l.by, bz = l.bz;
                l.tile_cells.assign(nb, kStgTile[0]);
                l.by.assign(nb, kStgTile[1]);
                l.bz.assign(nb, kStgTile[2]);
                e = build_list(ctx, 1);
                if (e != hipSuccess) break;
                const WorkList w = work_list(ctx, 1, -1);
                double ms = 0.0;
                e = timeit([&] { return launch_recon_mfma(ctx->user.recon_prec, gp32(ctx), w, ctx->Ntot, Q, G, L,
                                                          ctx->M, ctx->Kmf, ctx->P, ctx->gp, 0,
                                                          BlendIO{ctx->jump, ctx->mlp_packed, nullptr, nullptr},
                                                          false, true, s); },
                           ms);
                const cgks_launch stg{kStgTile[0], 0, 0, kStgTile[1], kStgTile[2], 1};
                note(1, stg, ms);
                if (ms < best) {
                    l.cfg = stg;
                } else {
                    l.tile_cells = tc;
                    l.by = by;
                    l.bz = bz;
                    e = build_list(ctx, 1);
                }
                if (e != hipSuccess) break;
            }
        }
        // 3) flux: XCD order (its inputs are the Gauss-point values of the reconstruction run
        //    just before)
        {
            cgks_ctx::List &l = ctx->wl[2];
            double best = 1e300;
            cgks_launch pick = l.cfg;
            e = run_recon(ctx, -1, Q, G, L, s);
            for (int x = 0; x < 2 && e == hipSuccess; ++x) {
                l.cfg.ngroups = 0;
                l.cfg.xcd = x;
                double ms = 0.0;
                e = timeit([&] { return run_flux(ctx, -1, dt_dev, Q, s); }, ms);
                note(2, l.cfg, ms);
                if (ms < best) {
                    best = ms;
                    pick = l.cfg;
                }
            }
            l.cfg = pick;
        }
        if (e != hipSuccess) rc = hip_fail(e, "autotune");
    } while (0);
    ctx->prof = saved_prof;
    ctx->pool.push_back(e0);
    ctx->pool.push_back(e1);
    ctx->stage1_done = false;
    return rc;
}

int cgks_step_graph(cgks_ctx *ctx, double *Q, double *G, double *L, double *dt_dev, int use_cfl, void *stream) {
    if (!ctx || !dt_dev || !Q || !G || !L) return fail(CGKS_EINVAL, "cgks_step_graph: NULL argument");
    const void *key[4] = {Q, G, L, dt_dev};
    const int cfl = use_cfl ? 1 : 0;
    bool same = ctx->gexec && ctx->gkey_cfl == cfl;
    for (int i = 0; i < 4 && same; ++i) same = ctx->gkey[i] == key[i];
    if (!same) {
        drop_graph(ctx);
        if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "capture stream");
        const bool saved_prof = ctx->prof;
        ctx->prof = false;
        HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        const int st = cgks_step(ctx, Q, G, L, dt_dev, use_cfl, ctx->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
        ctx->prof = saved_prof;
        if (st != CGKS_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != CGKS_OK ? st : hip_fail(e, "end capture");
        }
        ctx->graph = g;
        HIP_TRY(hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0), "instantiate graph");
        for (int i = 0; i < 4; ++i) ctx->gkey[i] = key[i];
        ctx->gkey_cfl = cfl;
    }
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(hipGraphLaunch(ctx->gexec, s), "graph launch");
    ctx->stage1_done = false;
    return CGKS_OK;
}

// ---- learned blend weights ---------------------------------------------------------------
static int mlp_upload(cgks_ctx *ctx, const float *w) {
    std::vector<unsigned char> packed(kMlpPackBytes);
    mlp_pack(w, packed.data());
    HIP_TRY(hipDeviceSynchronize(), "sync");
    HIP_TRY(hipMemcpy(ctx->mlp_w, w, sizeof(float) * kMlpParams, hipMemcpyHostToDevice), "upload MLP");
    HIP_TRY(hipMemcpy(ctx->mlp_packed, packed.data(), kMlpPackBytes, hipMemcpyHostToDevice), "upload MLP blocks");
    HIP_TRY(hipMemset(ctx->mlp_m, 0, sizeof(float) * kMlpParams), "clear Adam");
    HIP_TRY(hipMemset(ctx->mlp_v, 0, sizeof(float) * kMlpParams), "clear Adam");
    ctx->adam_t = 0;
    ctx->mlp_ready = true;
    drop_graph(ctx);
    return CGKS_OK;
}

int cgks_mlp_init(cgks_ctx *ctx, unsigned long long seed) {
    if (!ctx) return fail(CGKS_EINVAL, "cgks_mlp_init: NULL context");
    // splitmix64 stream -> uniform in [-1, 1)
    unsigned long long x = seed;
    auto next = [&]() {
        unsigned long long z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    };
    std::vector<float> w(kMlpParams, 0.0f);
    const double a1 = std::sqrt(6.0 / kMlpIn), a2 = std::sqrt(6.0 / kMlpHidden);
    for (int i = 0; i < kMlpHidden * kMlpIn; ++i) w[i] = (float)(a1 * next());
    for (int i = 0; i < kMlpOut * kMlpHidden; ++i) w[kMlpOffW2 + i] = (float)(a2 * next());
    return mlp_upload(ctx, w.data());
}

int cgks_mlp_set(cgks_ctx *ctx, const float *w, int n) {
    if (!ctx || !w) return fail(CGKS_EINVAL, "cgks_mlp_set: NULL argument");
    if (n != kMlpParams) return fail(CGKS_EINVAL, "cgks_mlp_set: n must be 839");
    return mlp_upload(ctx, w);
}

int cgks_mlp_get(cgks_ctx *ctx, float *w, int n) {
    if (!ctx || !w) return fail(CGKS_EINVAL, "cgks_mlp_get: NULL argument");
    if (n != kMlpParams) return fail(CGKS_EINVAL, "cgks_mlp_get: n must be 839");
    HIP_TRY(hipDeviceSynchronize(), "sync");
    HIP_TRY(hipMemcpy(w, ctx->mlp_w, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "read MLP");
    return CGKS_OK;
}

static int mlp_scratch(cgks_ctx *ctx, long B) {
    if (B <= ctx->mlp_scratch_n) return CGKS_OK;
    HIP_TRY(hipDeviceSynchronize(), "sync");
    (void)hipFree(ctx->mlp_scratch);
    ctx->mlp_scratch = nullptr;
    ctx->mlp_scratch_n = 0;
    HIP_TRY(hipMalloc((void **)&ctx->mlp_scratch, sizeof(float) * (size_t)mlp_scratch_floats((int)B)), "MLP scratch");
    ctx->mlp_scratch_n = B;
    return CGKS_OK;
}

int cgks_mlp_grad(cgks_ctx *ctx, const float *X, const float *T, long n, float *grad, float *loss, void *stream) {
    if (!ctx || !X || !T || !grad || !loss) return fail(CGKS_EINVAL, "cgks_mlp_grad: NULL argument");
    if (n < 1 || n > (1L << 26)) return fail(CGKS_EINVAL, "cgks_mlp_grad: n must be in [1, 2^26]");
    if (!ctx->mlp_ready) return fail(CGKS_EINVAL, "cgks_mlp_grad: no MLP parameters set");
    int st = mlp_scratch(ctx, n);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(launch_mlp_grad(ctx->mlp_w, X, T, n, 0, (int)n, ctx->mlp_scratch, grad, loss, s), "MLP gradient");
    return CGKS_OK;
}

int cgks_mlp_train(cgks_ctx *ctx, const float *X, const float *T, long n, int steps, int batch, float lr,
                   float *loss_hist, void *stream) {
    if (!ctx || !X || !T) return fail(CGKS_EINVAL, "cgks_mlp_train: NULL argument");
    if (n < 1 || steps < 0 || batch < 1 || batch > (1 << 24) || !(lr > 0.0f))
        return fail(CGKS_EINVAL, "cgks_mlp_train: need n >= 1, steps >= 0, 1 <= batch <= 2^24, lr > 0");
    if (!ctx->mlp_ready) return fail(CGKS_EINVAL, "cgks_mlp_train: no MLP parameters set");
    int st = mlp_scratch(ctx, batch);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    float *hist = nullptr;
    if (loss_hist && steps > 0) HIP_TRY(hipMalloc((void **)&hist, sizeof(float) * steps), "loss history");
    int rc = CGKS_OK;
    for (int k = 0; k < steps && rc == CGKS_OK; ++k) {
        const long first = (long)((long long)k * batch % n);
        hipError_t e = launch_mlp_grad(ctx->mlp_w, X, T, n, first, batch, ctx->mlp_scratch, ctx->mlp_g,
                                       hist ? hist + k : ctx->mlp_loss, s);
        if (e == hipSuccess)
            e = launch_mlp_adam(ctx->mlp_w, ctx->mlp_m, ctx->mlp_v, ctx->mlp_g, lr, 0.9f, 0.999f, 1e-8f, ++ctx->adam_t, s);
        if (e != hipSuccess) rc = hip_fail(e, "MLP training step");
    }
    if (hist) {
        if (rc == CGKS_OK) {
            hipError_t e = hipMemcpyAsync(loss_hist, hist, sizeof(float) * steps, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) rc = hip_fail(e, "loss history");
        } else {
            (void)hipStreamSynchronize(s);
        }
        (void)hipFree(hist);
    }
    if (rc) return rc;
    // refresh the inference blocks from the trained FP32 parameters
    std::vector<float> w(kMlpParams);
    std::vector<unsigned char> packed(kMlpPackBytes);
    HIP_TRY(hipStreamSynchronize(s), "sync");
    HIP_TRY(hipMemcpy(w.data(), ctx->mlp_w, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "read MLP");
    mlp_pack(w.data(), packed.data());
    HIP_TRY(hipMemcpy(ctx->mlp_packed, packed.data(), kMlpPackBytes, hipMemcpyHostToDevice), "upload MLP blocks");
    drop_graph(ctx);
    return CGKS_OK;
}

int cgks_mlp_infer(cgks_ctx *ctx, const float *X, long n, double *Y, void *stream) {
    if (!ctx || !X || !Y) return fail(CGKS_EINVAL, "cgks_mlp_infer: NULL argument");
    if (n < 0) return fail(CGKS_EINVAL, "cgks_mlp_infer: n must be >= 0");
    if (!ctx->mlp_ready) return fail(CGKS_EINVAL, "cgks_mlp_infer: no MLP parameters set");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(launch_mlp_infer(X, n, ctx->mlp_packed, Y, s), "MLP inference");
    return CGKS_OK;
}

int cgks_weights(cgks_ctx *ctx, const double *Q, const double *G, const double *L, float *X, double *Wt,
                 unsigned char *jump, void *stream) {
    if (!ctx || !Q || !G || !L || !X || !Wt) return fail(CGKS_EINVAL, "cgks_weights: NULL argument");
    if (ctx->user.recon_impl != 0 || ctx->user.recon_prec != 0 || gp32(ctx) || ctx->user.linear)
        return fail(CGKS_EUNSUPPORTED, "cgks_weights: FP64 nonlinear matrix-core contexts only");
    if (ctx->P.weights == 1 && !ctx->mlp_ready) return fail(CGKS_EINVAL, "learned weights: no MLP parameters set");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    HIP_TRY(launch_jump(work_list(ctx, 3, -1), ctx->Ntot, Q, ctx->P, ctx->jump, ctx->jcount, s), "jump");
    ctx->jexamined += ctx->Ntot;
    BlendIO io{ctx->jump, ctx->mlp_packed, Wt, X};
    HIP_TRY(launch_recon_mfma(0, false, work_list(ctx, 1, -1), ctx->Ntot, Q, G, L, ctx->M, ctx->Kmf, ctx->P, ctx->gp,
                              ctx->wl[1].cfg.ngroups, io, true, ctx->wl[1].cfg.stage != 0, s),
            "recon export");
    if (jump) HIP_TRY(hipMemcpyAsync(jump, ctx->jump, ctx->Ntot, hipMemcpyDeviceToDevice, s), "copy jump flags");
    return CGKS_OK;
}

int cgks_mlp_fallback(cgks_ctx *ctx, long long *flagged, long long *examined) {
    if (!ctx || !flagged || !examined) return fail(CGKS_EINVAL, "cgks_mlp_fallback: NULL argument");
    HIP_TRY(hipStreamSynchronize(ctx->last), "sync");
    unsigned long long f = 0;
    HIP_TRY(hipMemcpy(&f, ctx->jcount, sizeof f, hipMemcpyDeviceToHost), "read count");
    HIP_TRY(hipMemset(ctx->jcount, 0, sizeof f), "clear count");
    *flagged = (long long)f;
    *examined = ctx->jexamined;
    ctx->jexamined = 0;
    return CGKS_OK;
}

}  // extern "C"
