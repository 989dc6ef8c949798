/*
 * cgks.h — C ABI of the MI355X (gfx950) implementation of the per-stage path of the
 * fifth-order compact gas-kinetic scheme (CGKS-5) of Yang, Zhao & Xu, "An effective
 * implementation of high-order compact gas-kinetic scheme on structured meshes for
 * compressible flows".
 *
 * One context holds the mesh of one or more periodic structured blocks, their metrics
 * (Sec. 4: affine map to the standard cell, J0 and (J0^T)^-1; Sec. 2: 2x2 Gauss points
 * per quadrilateral face; Appendix: trilinear cell volume), the constant reconstruction
 * matrices of the standard cell (Sec. 3.3 eq. compact-big-5, Sec. 4 eq. compact-big-ref),
 * and the work buffers of a stage.  The caller owns the flow state.
 *
 * State layout (all blocks concatenated; per block SoA, x fastest, cell c = i + nx(j + ny k)):
 *   Q[5][N]      cell averages (rho, rho U, rho V, rho W, rho E)          (Sec. 2, eq. semi)
 *   G[5][3][N]   cell-averaged physical gradient d Q_v / d x_j            (Sec. 3.1, eq. derivative)
 *   L[5][12][N]  line derivatives in the reference frame: Q(G(s,+)) - Q(G(s,-)) along the
 *                12 lines joining paired face Gauss points                 (Sec. 3.1, eq. derivative-l)
 *                line s = 4q + k joins Gauss point k of the minus-q face to Gauss point k of
 *                the plus-q face; Gauss point k on a face of axis q has coordinates
 *                ((2(k&1)-1) g, (2(k>>1)-1) g) along the two other axes in ascending order,
 *                g = 1/(2 sqrt 3), on the face parametrised over [-1/2, 1/2]^2.
 * with N the total cell count.  Nodes of a block: (nx+1)(ny+1)(nz+1) x 3 doubles, x fastest;
 * the block is periodic and node index n along an axis is node 0 shifted by the period.
 *
 * Pointers: "device" pointers are HIP device allocations owned by the caller; "host"
 * pointers are ordinary host memory.  No call allocates on a stage or step; stage and step
 * never synchronise the stream, so a sequence of them can be captured into a HIP graph.
 * A context is bound to the device that was current at creation and is not thread-safe.
 *
 * Errors: every call returns a cgks_status.  Argument errors are detected on the host
 * before any device work.  Non-physical states met by the kernels (rho <= 0, p <= 0 or a
 * non-finite value at a Gauss point) set a device flag that cgks_check reports.  Nothing
 * aborts and nothing prints; cgks_last_error() gives a message for the last failure of the
 * calling thread.
 */
#ifndef CGKS_H
#define CGKS_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cgks_ctx cgks_ctx;

typedef enum {
    CGKS_OK = 0,
    CGKS_EINVAL = -1,        /* bad argument (detected on the host)                         */
    CGKS_EHIP = -2,          /* a HIP runtime call failed                                   */
    CGKS_ENOMEM = -3,        /* device allocation failed (context creation only)            */
    CGKS_ENONPHYS = -4,      /* non-physical state seen by a kernel (see cgks_check)        */
    CGKS_EUNSUPPORTED = -5   /* option not available in this build                          */
} cgks_status;

/* Scheme parameters.  Defaults (cgks_default_params) are the paper's constants:
 * gamma 1.4, CFL 0.5, inviscid collision time tau = tau_eps dt + tau_C |dp/sum p| dt with
 * tau_eps 0.05, tau_C 5 (Sec. 5); GENO eps 1e-15, r = 2 (Sec. 3.3). */
typedef struct {
    double gamma;
    double cfl;
    double tau_eps, tau_C;
    double mu0;          /* dynamic viscosity at T_ref (viscous mode)                       */
    double T_ref;        /* Sutherland reference temperature, in units of p/rho             */
    double S_suth;       /* Sutherland constant, same units                                 */
    double Pr;           /* Prandtl number (heat-flux correction when prandtl_fix = 1)      */
    double geno_C;       /* path-function constant of chi = tanh(C alpha)/tanh(C)           */
    double geno_eps;     /* epsilon of the smoothness ratios and linear weights             */
    double geno_r;       /* exponent r of the path function                                 */
    int viscous;         /* 0: inviscid collision time; 1: tau = mu/p + tau_C |dp/sum p| dt */
    int visc_law;        /* 0: constant mu0; 1: Sutherland                                  */
    int tau_zero;        /* 1: tau = 0, f = g0 (1 + A t) (accuracy test of Sec. 5.1)        */
    int linear;          /* 1: chi = 1 (linear CGKS-5)                                      */
    int prandtl_fix;     /* 1: heat-flux correction to Pr (viscous mode only)               */
    int recon_prec;      /* reconstruction contractions: 0 FP64 matrix cores; 1 FP32x3 split
                            precision on the FP32 matrix cores; 2 BF16x3 split precision on
                            the BF16 matrix cores (both with FP32 accumulation)             */
    int flux_prec;       /* gas-kinetic flux arithmetic: 0 FP64, 1 FP32.  Either reduced
                            option stores Gauss-point data in FP32; metrics, the time step
                            and the S2O4 accumulation of Q, G, L stay FP64                  */
    int recon_impl;      /* reconstruction kernel: 0 matrix cores (MFMA, default),
                            1 vector-ALU kernel (one thread per cell and variable),
                            2 per-cell stored matrices: the cell's coefficient map from its
                            physical-frame stencil data (34 x 84) and its Gauss-point
                            evaluation (96 x 34), built at context creation and read every
                            stage; 48,960 bytes per cell (the storage the shared standard
                            cell of Sec. 4 avoids).  1 and 2 are FP64 only              */
    int per_block;       /* multi-block launches: 0 one launch per kernel covering every
                            block (work list of tiles over all blocks, default); 1 one
                            launch per kernel and block (the comparison baseline)          */
    int weights;         /* blend weights: 0 GENO (Sec. 3.3); 1 learned (MLP, see below)
                            with GENO where the jump indicator fires.  1 needs the FP64
                            matrix-core reconstruction and the nonlinear scheme            */
    double jump_thresh;  /* jump indicator: max over face neighbours m of
                            |p_m - p_0| / (p_m + p_0) above this (default 0.05)            */
    int bc[6];           /* side types of every block, sides x-, x+, y-, y+, z-, z+:
                            0 periodic (default), 1 symmetry plane (slip, adiabatic),
                            2 no-slip adiabatic wall, 3 far field (the ghost data are the
                            uniform state farfield, and a far-field face takes the
                            gas-kinetic flux between the interior Gauss-point state and
                            it), 4 non-reflecting (Sec. 5, jet outflow sides: the ghost data
                            continue the cell beside the side linearly, its average plus its
                            reference gradient times the one-cell offset, its gradient
                            unchanged; a face on the side takes the gas-kinetic flux between
                            the interior Gauss-point state and the boundary state of locally
                            one-dimensional characteristics, the outgoing Riemann invariant
                            from the interior and the incoming one from farfield; EUNSUPPORTED
                            with learned weights).  The two sides of an axis are both periodic or both not.  Sec. 5 names walls but gives no
                            treatment for the compact stencil; here a neighbour behind a
                            wall is the mirror image of its mirror cell inside (average and
                            cell-averaged gradient reflected across the wall plane, with the
                            normal momentum, or at a no-slip wall every momentum component,
                            reversed) and a wall face takes the gas-kinetic flux between the
                            interior Gauss-point state and its mirror image; at a no-slip
                            wall the mass and energy components of F and F_t are zero.
                            A wall side must be a plane normal to its axis, the axis pointing
                            into the block, and the two sides of the axis must share their
                            tangential node coordinates (EINVAL at creation otherwise).
                            Walls need recon_impl 0 (EUNSUPPORTED).  With learned weights
                            the jump indicator takes a neighbour behind a wall as the cell's
                            mirror image and one behind a far-field side as the far field */
    double farfield[5];  /* far-field state (rho, rho U, rho V, rho W, rho E) of bc 3 and 4 sides;
                            positive density and pressure (EINVAL otherwise)             */
    int positivity;      /* 1: interface-state limiter (not in the paper; for flows whose
                            local Mach number reaches ~3, where internal energy is a small
                            part of the total): at each face Gauss point, a cell's
                            reconstructed state (value q, gradient g) becomes
                            qbar + theta (q - qbar) and theta g, theta the largest value in
                            [0, 1] keeping its density and pressure at or above pos_eps times
                            the cell average qbar's own.  Periodic blocks only (EUNSUPPORTED
                            with wall sides).  Default 0                                 */
    double pos_eps;      /* floor of the limiter, in (0, 1) (default 1e-3)               */
} cgks_params;

/* Fill *p with the defaults listed above (inviscid, nonlinear, FP64). */
void cgks_default_params(cgks_params *p);

/* Create a context on the current device.
 *   nblocks      number of periodic blocks (>= 1)
 *   dims         host, nblocks*3 ints: nx, ny, nz of each block (each >= 1)
 *   nodes        host, nblocks pointers, each to (nx+1)(ny+1)(nz+1)*3 doubles (x fastest)
 *   p            host, scheme parameters (copied)
 *   stream       hipStream_t used for the set-up work (may be NULL: the null stream)
 * Metrics are computed on the device.  Cells must have positive volume and positive
 * det J0.  The total number of cells must be below 2^27 (the kernels index one component
 * array with 32-bit offsets; one MI355X holds about 33M cells of state and buffers).  The
 * internal Gauss-point buffer pads a block's rows to a multiple of 16 cells where that costs
 * at most a quarter more (aligned stores), so its size grows by up to 25 % for blocks whose x
 * extent is not a multiple of 16.  On failure *out is NULL. */
int cgks_ctx_create(cgks_ctx **out, int nblocks, const int *dims, const double *const *nodes,
                    const cgks_params *p, void *stream);

/* Release every device buffer of the context (synchronises the device).  NULL is a no-op. */
void cgks_ctx_destroy(cgks_ctx *ctx);

/* Flow diagnostics of the Taylor-Green section (Sec. 5) over all cells of all blocks:
 *   E_k   = 1/(rho0 |Omega|) int rho U.U / 2 dV      (volume-averaged kinetic energy)
 *   eps_S = 1/(rho0 |Omega|) int mu |curl U|^2 dV     (integrated enstrophy)
 * by the midpoint rule over the cells, from the cell averages Q and the cell-averaged
 * gradients G (layouts of cgks_stage).  rho0 is the mean density (conserved by the scheme);
 * the velocity gradient of a cell is (grad(rho U) - U grad rho) / rho; mu follows the
 * viscosity law of the parameters at T = p / rho (mu0 when visc_law is 0).
 *   out   device, 6 doubles: E_k, eps_S, mean rho, mean rho E, min rho, min p
 * Deterministic (a fixed partition of the cells and a fixed summation tree); asynchronous on
 * stream; errors: CGKS_EINVAL for NULL arguments. */
int cgks_diagnostics(cgks_ctx *ctx, const double *Q, const double *G, double *out, void *stream);

/* Q-criterion of every cell, the vortex-identification field of the Taylor-Green section
 * (Sec. 5): q = (|Omega|^2 - |S|^2) / 2 with S, Omega the symmetric and antisymmetric parts of
 * the velocity gradient (Frobenius norms), the velocity gradient of a cell being
 * (grad(rho U) - U grad rho) / rho from its cell averages and cell-averaged gradients.
 * Q [5][N], G [5][3][N]: device state; out: device array of N doubles, overwritten.
 * Enqueued on `stream`; EINVAL on a NULL argument. */
int cgks_qcriterion(cgks_ctx *ctx, const double *Q, const double *G, double *out, void *stream);

/* The diagnostics of cgks_diagnostics from the compact reconstruction (Sec. 5, Taylor-Green
 * vortex, with the velocity derivatives taken from the reconstruction at quadrature points):
 * each cell is integrated by 3^3 Gauss points of its trilinear map (volume element |det J|),
 * with the conserved variables and their gradients at the points from the cell's
 * reconstruction blended as at the face Gauss points, Q = chi P^4 + (1 - chi)(Q_0 + bbar . xi)
 * (eq. weno-new), reference gradients likewise, physical ones by (J0^T)^-1.  Converges at
 * fourth order or better on smooth fields (the midpoint rule of cgks_diagnostics: second).
 * Q, G, L: device state; out: device array of 6 doubles, written on the stream, as for
 * cgks_diagnostics (minima over the quadrature points).  Periodic blocks only
 * (CGKS_EUNSUPPORTED with wall sides; at most 1024 blocks); deterministic; overwrites the
 * context's Gauss-point buffer (no stage needs it across calls).  EINVAL on a NULL argument. */
int cgks_diagnostics_hq(cgks_ctx *ctx, const double *Q, const double *G, const double *L, double *out,
                        void *stream);

/* Total number of cells N of the context. */
long cgks_num_cells(const cgks_ctx *ctx);

/* Global time step by the CFL condition of Sec. 5: dt = CFL / max over cells of
 * sum_d (|U.n_d| + c)/h_d (h_d = volume / mean area of the two d-faces, n_d their mean
 * normal), and in viscous mode also CFL h_min^2 / (3 nu).  Q: device [5][N];
 * dt_dev: device, one double, written on the stream. */
int cgks_dt(cgks_ctx *ctx, const double *Q, double *dt_dev, void *stream);

/* cgks_dt for callers that cannot allocate device memory at call time (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same result, bitwise (the
 * same partition of the cells into partial minima), with the partial minima in a static
 * device array of the library (1024 doubles, 8 KB per GPU, held until the process ends)
 * instead of context memory.  It launches two kernels and calls no hipMalloc, hipFree or
 * other allocating routine; nothing needs clearing (every partial is written before it is
 * read).  Every call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other contexts, other threads) race and must be ordered by the caller.  Q, dt_dev
 * and stream as for cgks_dt.  Errors: CGKS_EINVAL for a NULL argument or a context whose
 * partition needs more than 1024 partial minima (never, for partitions of at most 1024
 * workgroups, which the context uses); CGKS_EHIP if the array's address could not be
 * looked up on this device when the context was created. */
int cgks_dt_noalloc(cgks_ctx *ctx, const double *Q, double *dt_dev, void *stream);

/* One S2O4 stage in place (temporal-discretisation section of the paper).
 *   stage 1: Q* = Q + dt/2 L(Q) + dt^2/8 dL/dt;  G*, L* from the interface values evolved to
 *            t + dt/2; saves what stage 2 needs in the context.
 *   stage 2: Q = Q^n + dt L(Q^n) + dt^2/6 (dL/dt(Q^n) + 2 dL/dt(Q*));  G, L from the
 *            interface values at t^n evolved over dt with the stage-2 time derivative.
 * dt_dev: device double (the same value for both stages).  Q, G, L: device state.
 * Stage 2 must follow a stage 1 on the same context with the same dt. */
int cgks_stage(cgks_ctx *ctx, int stage, const double *dt_dev, double *Q, double *G, double *L,
               void *stream);

/* One full S2O4 step: if use_cfl, dt is computed into *dt_dev first (cgks_dt); otherwise
 * *dt_dev is used as given.  Then stage 1 and stage 2. */
int cgks_step(cgks_ctx *ctx, double *Q, double *G, double *L, double *dt_dev, int use_cfl,
              void *stream);

/* Synchronise the context's last stream and report the device error flag:
 * *flags_host = 0 if clean, else a bit mask (1: rho <= 0, 2: p <= 0, 4: non-finite).
 * Returns CGKS_ENONPHYS if a flag is set (and clears it), CGKS_OK otherwise. */
int cgks_check(cgks_ctx *ctx, int *flags_host);

/* Gauss-point reconstruction of the whole state (test and diagnostics entry point):
 * gp: device [N][24][5][4], per cell the value and physical gradient of every conserved
 * variable at its 24 face Gauss points (face m = 2q+s, point k, index 4m+k). */
int cgks_recon(cgks_ctx *ctx, const double *Q, const double *G, const double *L, double *gp,
               void *stream);

/* Gas-kinetic flux (Sec. 2, eq. flux and its time linearisation) at n independent points.
 * Device arrays: ql, qr [n][5]; gl, gr [n][5][3] (physical gradients); nrm [n][3] unit
 * normals pointing from left to right; dt_dev one double.  Outputs (device): F, Ft [n][5]
 * (flux and its time derivative per unit area); sides [n][4][5] = (Q^l, dQ^l/dt, Q^r,
 * dQ^r/dt) one-sided interface values.  Non-physical input sets the device flag of ctx. */
int cgks_flux(cgks_ctx *ctx, long n, const double *ql, const double *gl, const double *qr,
              const double *gr, const double *nrm, const double *dt_dev, double *F, double *Ft,
              double *sides, void *stream);

/* Per-cell metrics computed at creation (test entry point).  Device outputs, any may be
 * NULL: vol [N]; J0 [N][9] row-major dx_i/dxi_j; fn [N][3][4][3] unit normals of the three
 * plus faces; fw [N][3][4] Gauss weight times area element. */
int cgks_metrics(cgks_ctx *ctx, double *vol, double *J0, double *fn, double *fw, void *stream);

/* Kernel timing (tracing aid).  When enabled, every kernel launch of cgks_dt / cgks_stage is
 * bracketed by HIP events recorded on the caller's stream; cgks_profile_read synchronises and
 * returns, per kernel kind, the summed elapsed milliseconds and the launch count since the
 * last read, then resets them.  Kinds: 0 dt, 1 reconstruction (both stages), 2 flux of stage 1,
 * 3 update of stage 1, 4 flux of stage 2, 5 update of stage 2 (the two stages' flux and update
 * kernels do different work).  Not for use under HIP graph capture.  ms and launches: host
 * arrays of CGKS_NKINDS. */
#define CGKS_NKINDS 6
int cgks_profile(cgks_ctx *ctx, int enable);
int cgks_profile_read(cgks_ctx *ctx, double *ms, long *launches);

/* ---- Multi-block launches, autotuning and graph replay ------------------------------------
 * The reconstruction, flux and update kernels walk a work list of tiles (runs of consecutive
 * cells of one block) that spans every block, so one launch per kernel advances the whole
 * multi-block mesh.  Launch configuration per kernel kind (1 reconstruction, 2 flux, 3 update):
 *   tile_cells  cells per tile.  Reconstruction: a multiple of 16 in [16, 4096] (one
 *               workgroup of 8 waves takes a tile and first stages the constant matrices in
 *               LDS; a wave takes 16 cells of one variable).  Default: bricks of 16 x 8 x 10
 *               cells staged in LDS (stage 1) for the FP64 and FP32x3 reconstruction, runs of
 *               1536 cells for BF16x3;
 *               flux 128 and update 256 are fixed by their workgroup size.
 *   ngroups     0: one workgroup per unit (tile, or tile and Gauss point for the flux);
 *               > 0: a persistent grid of that many workgroups striding over the units
 *               (reconstruction and update; the flux takes 0 only).
 *   xcd         1: the workgroups on XCD x (w mod 8 == x) walk the x-th contiguous eighth of
 *               the units (a persistent grid must then be a multiple of 8); 0: plain order.
 * The arithmetic of a cell does not depend on the configuration: results are bitwise equal
 * for every choice. */
typedef struct {
    int tile_cells;
    int ngroups;
    int xcd;
    int brick_y, brick_z;  /* reconstruction only: 0, 0 for runs of tile_cells cells; both > 0 for
                              bricks of tile_cells x brick_y x brick_z cells (clipped to the
                              block) whose workgroup walks its planes in order of z */
    int stage;             /* reconstruction only: 1 stages each brick with its one-cell halo in
                              LDS, one conserved variable at a time, and gathers the neighbours
                              from there; needs bricks with tile_cells = 16 and
                              (brick_y + 2) (brick_z + 2) <= 120, and the FP64 or FP32x3
                              reconstruction.  0: neighbours gathered from memory */
} cgks_launch;

/* Read the launch configuration of a kernel kind (1, 2 or 3) into *out (host). */
int cgks_get_launch(const cgks_ctx *ctx, int kind, cgks_launch *out);

/* Set the launch configuration of a kernel kind (host, copied).  Rebuilds the work list on
 * the device (synchronises the device); not for use under HIP graph capture. */
int cgks_set_launch(cgks_ctx *ctx, int kind, const cgks_launch *cfg);

/* Autotuner: times candidate configurations of the reconstruction (runs or bricks per
 * block-size class: blocks below 2^17 cells, below 2^19, and larger; then grid and XCD order) and of the
 * flux (XCD order) on the given state with HIP events, and keeps the fastest.
 * Q, G, L, dt_dev: device state and time step (read only; the stage buffers of the context
 * are overwritten).  reps: timed launches per candidate (>= 1).  report: host array of at
 * least report_len doubles or NULL; receives per candidate (kind, tile_cells, ngroups, xcd,
 * brick_y, brick_z, ms), preceded by the number of candidates.  Synchronises the stream; not capturable. */
int cgks_autotune(cgks_ctx *ctx, const double *Q, const double *G, const double *L, const double *dt_dev,
                  int reps, double *report, int report_len, void *stream);

/* One S2O4 step as cgks_step, replayed from a HIP graph of [dt,] stage 1 and stage 2 that the
 * context captures on first use and captures again when Q, G, L, dt_dev or use_cfl change.
 * Launches the graph on `stream`.  Capture allocates the graph (once); replays allocate
 * nothing.  Profiling events are not recorded for graph replays. */
int cgks_step_graph(cgks_ctx *ctx, double *Q, double *G, double *L, double *dt_dev, int use_cfl,
                    void *stream);

/* ---- Learned blend weights ---------------------------------------------------------------
 * An MLP 18 -> 32 (ReLU) -> 7 stands in for the nonlinear weights of Sec. 3.3: output 0 gives
 * chi through a sigmoid, outputs 1..6 the weights omega_m of the six linear sub-polynomials
 * through a softmax.  Inputs per cell and conserved variable: the 6 face-neighbour differences
 * Q_{1,m} - Q_0 (m = 2q + s) and the 12 line derivatives L_s, divided by (their largest
 * magnitude + 1e-12).  Parameters: FP32, 839 values W1[32][18], b1[32], W2[7][32], b2[7].
 * Inference inside the reconstruction runs in BF16 on the matrix cores (FP32 accumulation);
 * training runs in FP32 (mean over the batch of the squared error of the 7 outputs, Adam
 * with beta1 0.9, beta2 0.999, eps 1e-8).  Feature and target arrays are device FP32,
 * row-major [n][18] and [n][7]. */
#define CGKS_MLP_PARAMS 839

/* Initialise the parameters from a seed (uniform He initialisation, zero biases) and reset
 * the Adam moments.  Synchronous. */
int cgks_mlp_init(cgks_ctx *ctx, unsigned long long seed);

/* Set / read the FP32 parameters (host arrays of n = CGKS_MLP_PARAMS).  Setting resets the
 * Adam moments.  Synchronous. */
int cgks_mlp_set(cgks_ctx *ctx, const float *w, int n);
int cgks_mlp_get(cgks_ctx *ctx, float *w, int n);

/* Gradient of the mean squared error over the n samples (X [n][18], T [n][7], device FP32)
 * into grad (device, CGKS_MLP_PARAMS floats) and loss (device, 1 float).  Allocates a
 * scratch of 72 n floats on first use (grows as needed). */
int cgks_mlp_grad(cgks_ctx *ctx, const float *X, const float *T, long n, float *grad, float *loss,
                  void *stream);

/* `steps` Adam steps with batches of `batch` samples taken in order, wrapping around the n
 * samples (step k uses samples k*batch .. k*batch+batch-1 mod n).  loss_hist: host array of
 * `steps` floats for the batch losses, or NULL.  Synchronises the stream when loss_hist is
 * given. */
int cgks_mlp_train(cgks_ctx *ctx, const float *X, const float *T, long n, int steps, int batch, float lr,
                   float *loss_hist, void *stream);

/* BF16 inference of the current parameters on given features: Y [n][7] device doubles
 * (chi, omega_1..6), exactly as the reconstruction evaluates them. */
int cgks_mlp_infer(cgks_ctx *ctx, const float *X, long n, double *Y, void *stream);

/* Reconstruction of the state that also reports, per cell and variable (sample index
 * 5 c + v), the learned-weight input features X [N*5][18] (device FP32), the blend weights
 * used Wt [N*5][7] (device doubles: chi, omega_1..6) and the jump flags jump [N] (device
 * bytes, may be NULL).  FP64 contexts with the nonlinear scheme only. */
int cgks_weights(cgks_ctx *ctx, const double *Q, const double *G, const double *L, float *X, double *Wt,
                 unsigned char *jump, void *stream);

/* Cells flagged by the jump indicator and cells examined since the last call (host outputs;
 * synchronises the stream). */
int cgks_mlp_fallback(cgks_ctx *ctx, long long *flagged, long long *examined);

/* Message of the last failing call on this thread ("" if none). */
const char *cgks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CGKS_H */
