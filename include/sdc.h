/*
 * sdc.h -- C ABI of the MI355X (gfx950) diagonal IMEX SDC library for the rotating
 * shallow-water equations in spherical-harmonic vorticity/divergence/geopotential form.
 *
 * Method: Freese, Goetschel, Lunet, Ruprecht, Schreiber, "Parallel performance of shared
 * memory parallel spectral deferred corrections".  The interface follows the paper's
 * initial-value problem u' = f_I(u) + f_E(u) (Section 4) and the three routines the paper
 * asks of a code that adopts diagonal SDC (Section 4.2): evaluate f_E, evaluate f_I, and solve
 * u - alpha f_I(u) = beta.  sdc_step is Algorithm 2 (diagonal IMEX SDC step) with the node
 * update of Section 4.2 and the MIN-SR-FLEX coefficients; the shallow-water split is the one
 * of Sections 3.2 and 4.4 (gravity-wave part L_g implicit, Coriolis plus nonlinear terms
 * explicit).
 *
 * ---------------------------------------------------------------------------------------------
 * Data layout (all buffers passed to the library are DEVICE pointers owned by the caller):
 *
 *   spectral field : ncoef complex128 values, interleaved (Re, Im) doubles, ncoef = (T+1)(T+2)/2,
 *                    m-major triangular: index(m, n) = m(2T+3-m)/2 + (n - m), 0 <= m <= n <= T.
 *                    Coefficients are of orthonormal spherical harmonics (integral over
 *                    mu in [-1,1] of Pbar_n^m squared is 1, no Condon-Shortley phase); only
 *                    m >= 0 is stored and a real field is f = sum_m s_m Re(F_m e^{i m lambda}),
 *                    s_0 = 1, s_m = 2.  Imaginary parts of m = 0 coefficients are ignored on
 *                    input by the transforms and are zero on output of every transform.
 *   state          : [batch][3][ncoef] spectral fields in the order (Phi', zeta, delta):
 *                    geopotential perturbation [m^2/s^2], vorticity [1/s], divergence [1/s]
 *                    (the solution vector of Section 3.2).
 *   grid field     : [batch][nlat][nlon] doubles; latitude index j runs north to south over the
 *                    Gauss-Legendre latitudes (mu_j = sin(latitude) descending), longitude
 *                    index i at lambda_i = 2 pi i / nlon.
 *
 * Execution: every call is enqueued on the HIP stream given to sdc_init and returns without
 * waiting for the GPU.  Argument errors are detected on the host before anything is enqueued
 * and returned synchronously (nothing is modified then).  Device-side conditions (non-finite
 * values produced by sdc_step) are reported by the next sdc_sync.  Device memory is allocated
 * by sdc_init and, once per handle, by the first call of an entry point that says so (adjoint,
 * comparison integrators); sdc_free releases everything the handle owns.  A handle must be used
 * from one host thread at a time; different handles are independent.  No C++ exception crosses
 * this interface.  With the environment variable SDC_ROCTX set (and not "0") when a handle is
 * created, its step phases are marked by host-side roctx ranges ("sdc.step", "sdc.f_E",
 * "sdc.f_E+update", "sdc.update") for rocprofv3 --marker-trace.
 * ---------------------------------------------------------------------------------------------
 */
#ifndef SDC_MI355X_H
#define SDC_MI355X_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SDC_OK = 0,
    SDC_EINVAL = -1,          /* invalid argument (message in sdc_last_error) */
    SDC_ENOMEM = -2,          /* device allocation failed */
    SDC_EHIP = -3,            /* a HIP runtime call failed */
    SDC_ENONFINITE = -4,      /* sdc_step produced a non-finite value (reported by sdc_sync) */
    SDC_EUNSUPPORTED = -5     /* valid but unsupported configuration (e.g. nlon not 2^p or 3*2^p) */
} sdc_status;

/* Arithmetic of the Legendre contractions (the only dense contraction of the step).  Gauss
 * nodes and weights, Legendre tables, Q, Q_Delta and the implicit-solve coefficients are
 * always generated and kept in FP64. */
typedef enum {
    SDC_FP64 = 0,             /* FP64 MFMA, FP64 tables */
    SDC_FP32_MFMA = 1,        /* FP32 MFMA (16x16x4) on FP32-rounded copies of the FP64 tables, the
                                 spectral / Fourier columns rounded to FP32 as they enter the MFMA,
                                 FP32 accumulation; every other step of sdc_step stays FP64 */
    SDC_BF16X3_MFMA = 2       /* the FP32 mode's operands (FP32 tables and columns), each split
                                 exactly into three BF16 terms on chip; every MFMA product is the
                                 sum of the 8 cross terms but the smallest (a2 b2, below 2^-32 |ab|)
                                 on BF16 MFMA (16x16x32), accumulated in FP32; every other step of
                                 sdc_step stays FP64 (Section 3.2's transforms; the compensated
                                 precision mode of the contractions) */
} sdc_precision;

typedef struct {
    int T;                    /* triangular truncation, 1 <= T <= 1023 */
    int nlat;                 /* Gaussian latitudes: even, nlat >= T+1 */
    int nlon;                 /* longitudes: nlon >= 2T+1 and nlon = 2^p or 3*2^p, nlon <= 2048 */
    double radius;            /* a [m] */
    double gravity;           /* g [m/s^2] */
    double omega;             /* Omega [1/s], Coriolis parameter f = 2 Omega mu */
    double mean_depth;        /* H [m]; mean geopotential Phi_bar = g H */
    int M;                    /* largest number of collocation nodes used by sdc_step, 1..8 */
    int K;                    /* largest number of sweeps used by sdc_step, 1..16 */
    int nodes;                /* collocation nodes: 0 = Radau-right (tau_M = 1), the only choice */
    int qdelta;               /* diagonal coefficients of the implicit sweeps (Section 4.2):
                                 0 = MIN-SR-FLEX, tau_m / min(s, M) in sweep s (the paper's choice);
                                 1 = MIN-SR-NS, tau_m / M in every sweep (a variant of the family:
                                 Q - Q_Delta is nilpotent);
                                 2 = parallel implicit Euler, tau_m in every sweep (another of the
                                 nonzero diagonals the node update admits) */
    int precision;            /* an sdc_precision value */
    int batch;                /* ensemble members sharing this truncation, >= 1 */
    int implicit_coriolis;    /* which terms are implicit (the change of split the paper's outlook
                                 names, Section 6): 0 = the paper's spectral split, f_I = L_g,
                                 f_E = L_c + N_a + N_r; 1 = the linear Coriolis term implicit too,
                                 f_I = L_g + L_c, f_E = N_a + N_r, the solve of u - alpha f_I(u) =
                                 beta then coupling the degrees n +- 1 of each order (two complex
                                 tridiagonal chains per order m).  With 1, sdc_step[_graph],
                                 eval_explicit, eval_implicit and imex_solve follow the new split;
                                 the adjoint, taped, sequential, IMEX-o2, group and one-node-per-
                                 launch paths return SDC_EUNSUPPORTED. */
} sdc_config;

typedef struct sdc_ctx* sdc_handle;

typedef struct {
    int T, nlat, nlon, ncoef, M, K, batch, precision;
    long long device_bytes;   /* device memory owned by the handle */
    long long table_bytes;    /* of which Legendre tables (all precisions kept) */
} sdc_info;

/* Create a handle: validates cfg, allocates every workspace, and generates on the GPU in FP64
 * the Gauss-Legendre latitudes and weights, the orthonormal Legendre functions Pbar_n^m and
 * H_n^m = (1-mu^2) dPbar_n^m/dmu at the northern latitudes (equatorial symmetry gives the
 * southern ones), the Radau-right nodes and collocation matrices Q for every node count
 * 1..cfg->M (Sections 4.1 and 4.2), and the FFT twiddles.  Blocks until setup is complete.
 * hip_stream: a hipStream_t (NULL = the default stream) on which every later call enqueues.
 * Returns SDC_EINVAL for an invalid cfg or out == NULL, SDC_EUNSUPPORTED for valid but
 * unsupported grids, SDC_ENOMEM / SDC_EHIP on device failures (nothing is leaked). */
int sdc_init(const sdc_config* cfg, void* hip_stream, sdc_handle* out);

/* Release the handle (waits for its stream first).  NULL is accepted. */
int sdc_free(sdc_handle h);

/* One diagonal IMEX SDC step (Algorithm 2) in place: state holds u_n on entry and u_{n+1} on
 * exit, for all batch members.  M nodes (1 <= M <= cfg.M) and K sweeps (1 <= K <= cfg.K);
 * sweeps 1..K-1 update all M nodes from the previous sweep's values, sweep K only the last
 * node; MIN-SR-FLEX coefficient of sweep s is tau_m / min(s, M).  dt > 0 and finite. */
int sdc_step(sdc_handle h, double* state, double dt, int M, int K);

/* Same result as sdc_step, executed as one hipGraph launch on the handle's stream.  The first
 * call for a given (state pointer, dt, M, K) captures the step's kernel sequence (on a private
 * stream) and instantiates it; later calls with the same key replay it.  A handle keeps the 8 most
 * recent graphs.  The state must stay allocated while a graph for it is cached. */
int sdc_step_graph(sdc_handle h, double* state, double dt, int M, int K);

/* One step of the sequential IMEX SDC of Algorithm 1 (node update of Section 4.1), the method dSDC
 * parallelises: K sweeps, each updating the M nodes one after another with backward-Euler
 * differences of f_I (weights dtau_j, dtau_1 = tau_1, dtau_j = tau_j - tau_{j-1}) and forward-Euler
 * differences of f_E (weights dtau_{j+1}) against the previous sweep; initial guess u_n at every
 * node; u_{n+1} = u_M^K.  1 + K M - 1 f_E evaluations per step, each over the batch members of one
 * node (dSDC evaluates all nodes of a sweep at once).  Same arguments, layouts and errors as
 * sdc_step; qdelta does not apply.  The first call allocates 4 M states per member of workspace.
 * sdc_step_sequential_graph: the same step as a cached hipGraph. */
int sdc_step_sequential(sdc_handle h, double* state, double dt, int M, int K);
int sdc_step_sequential_graph(sdc_handle h, double* state, double dt, int M, int K);

/* One step of IMEX-o2, the paper's reference integrator (Section 3.2): a Strang splitting with
 * Crank-Nicolson half steps for f_I = L_g around one Heun (explicit second-order Runge-Kutta)
 * step for f_E (the paper leaves the order open; the Crank-Nicolson part takes the half steps):
 *   u* = C(dt/2) u_n,  k1 = f_E(u*),  k2 = f_E(u* + dt k1),  u_{n+1} = C(dt/2)(u* + dt/2 (k1 + k2)),
 *   C(h) u = (I - h/2 L_g)^{-1} (I + h/2 L_g) u, closed form per coefficient.
 * In place on state [batch][3][ncoef], all members; dt > 0 and finite.  Two f_E evaluations per
 * step, in the handle's precision mode.  The first call on a handle allocates three states per
 * member of workspace; later calls allocate nothing.  Non-finite results are reported by sdc_sync.
 * imex2_step_graph: the same step as a cached hipGraph (as sdc_step_graph, keyed by state and dt). */
int imex2_step(sdc_handle h, double* state, double dt);
int imex2_step_graph(sdc_handle h, double* state, double dt);

/* For callers that cannot allocate device memory during the call (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same IMEX-o2 step as imex2_step, the
 * same kernels and bitwise the same result, with u*, k1 and k2 held in a fixed device array of the
 * library (64 MiB per device, reserved from library load until the process ends) instead of
 * handle workspaces allocated by the first imex2_step.  It allocates nothing and records no timing
 * events.  Needs 3 * batch * 3 * ncoef * 16 bytes (T255 with one member: 4.7 MB); SDC_EINVAL when
 * that exceeds 64 MiB (nothing enqueued), SDC_EHIP if the array's device address could not be
 * resolved at sdc_init.  Every handle on one device shares that device's array, and every value in
 * it is written before it is read within one call: calls that overlap on one device (other
 * streams or host threads) race and must be ordered by the caller. */
int imex2_step_noalloc(sdc_handle h, double* state, double dt);

/* Adjoint of one step: lam_n = (d u_{n+1} / d u_n)^T lam_np1 for the step taken from state_n
 * with the same dt, M, K (the step is recomputed internally from state_n, keeping the grid fields
 * of every stage; then the sweep runs in reverse with Q^T, the transposed per-degree solve and
 * the transposed transforms).  The inner product is the real Euclidean one over (Re, Im) of every
 * stored coefficient; imaginary parts of m = 0 entries of lam_n are set to zero.  lam_n may alias
 * lam_np1 but not state_n.  The first call on a handle allocates its adjoint workspaces
 * (grid fields of 1+(K-1)M stage states per member); later calls allocate nothing. */
int sdc_step_adjoint(sdc_handle h, const double* state_n, const double* lam_np1, double* lam_n,
                     double dt, int M, int K);

/* Taped adjoint (no recomputation; for callers that keep every step's stages, e.g. a whole
 * trajectory in HBM): sdc_step_taped is sdc_step that also writes the grid fields of every f_E
 * evaluation of the step (zeta, Phi', U, V at every grid point of the 1 + (K-1) M stage states of
 * each member) into `tape`, a caller-owned, 16-byte aligned device buffer of sdc_tape_size(h, M, K)
 * bytes;
 * sdc_step_adjoint_taped then computes the same lam_n as sdc_step_adjoint for that step from the
 * tape, skipping the forward recomputation.  The tape must come from a taped step of the same
 * handle with the same dt, M, K and stay unchanged until the adjoint call has run (stream order).
 * lam_n may alias lam_np1.  sdc_tape_size: SDC_EINVAL for M, K outside the configured ranges. */
int sdc_tape_size(sdc_handle h, int M, int K, long long* bytes);
int sdc_step_taped(sdc_handle h, double* state, double dt, int M, int K, void* tape);
int sdc_step_adjoint_taped(sdc_handle h, const void* tape, const double* lam_np1, double* lam_n,
                           double dt, int M, int K);

/* Scalar spherical-harmonic analysis of `batch` grid fields: grid [batch][nlat][nlon] ->
 * spec [batch][ncoef] (Gauss quadrature of the longitude Fourier coefficients truncated to
 * m <= T).  Exact inverse of sht_inverse on band-limited fields. */
int sht_forward(sdc_handle h, const double* grid, double* spec);

/* Scalar spherical-harmonic synthesis: spec [batch][ncoef] -> grid [batch][nlat][nlon]. */
int sht_inverse(sdc_handle h, const double* spec, double* grid);

/* Transpose of sht_inverse (real inner products of grid values and of (Re, Im) coefficient pairs):
 * spec = S^T grid, spec_nm = s_m sum_j Pbar_n^m(mu_j) sum_i grid_ij e^{-i m lambda_i}; imaginary
 * parts of m = 0 entries are zero.  Used for gradients of grid losses. */
int sht_inverse_adjoint(sdc_handle h, const double* grid, double* spec);

/* The solver of Section 4.2: u with u - alpha f_I(u) = beta, for states [batch][3][ncoef];
 * closed form per coefficient (with implicit_coriolis: the two tridiagonal chains per order).
 * u may alias beta.  alpha >= 0 and finite. */
int imex_solve(sdc_handle h, double alpha, const double* beta, double* u);

/* f_E(u) = L_c + N_a + N_r (Coriolis and nonlinear terms, Sections 3.2 and 4.4) for states
 * [batch][3][ncoef] by a transform round trip; fE must not alias u.  With implicit_coriolis,
 * N_a + N_r only (the products with the relative vorticity instead of the absolute one). */
int eval_explicit(sdc_handle h, const double* u, double* fE);

/* f_I(u) = L_g(u) (gravity-wave part, Section 3.2) for states [batch][3][ncoef]; fI may alias u.
 * With implicit_coriolis, L_g(u) + L_c(u), and fI must not alias u (SDC_EINVAL). */
int eval_implicit(sdc_handle h, const double* u, double* fI);

/* Wait for all work enqueued by this handle; returns SDC_ENONFINITE if any sdc_step since the
 * previous sdc_sync produced a non-finite value (and clears that condition), SDC_EHIP if the
 * stream reported an error. */
int sdc_sync(sdc_handle h);

/* Kernel classes of one step, for sdc_timing_read. */
typedef enum {
    SDC_KERNEL_SYNTHESIS = 0,   /* Legendre synthesis (spectral -> Fourier), MFMA */
    SDC_KERNEL_GRID = 1,        /* inverse FFT, grid products, forward FFT */
    SDC_KERNEL_ANALYSIS = 2,    /* Legendre analysis (Fourier -> spectral tendencies), MFMA */
    SDC_KERNEL_UPDATE = 3,      /* node integral + implicit solve; layout conversion of u_n */
    SDC_KERNEL_CLASSES = 4
} sdc_kernel_class;

/* Benchmark timing: while enabled, every kernel launch of the step is bracketed by a pair of
 * HIP events recorded on the handle's stream.  Enabling (on = 1) or disabling clears the
 * accumulated figures.  sdc_timing_read waits for the stream and returns, for one kernel class,
 * the summed event-measured duration in milliseconds and the number of launches. */
int sdc_timing_enable(sdc_handle h, int on);
int sdc_timing_read(sdc_handle h, int kernel_class, double* total_ms, long long* launches);

/* Read-before-write check (race detection for tests): while on = 1, the step (sdc_step,
 * sdc_step_graph, sdc_step_taped and the adjoint's recomputation) fills every workspace a launch
 * writes -- the Fourier fields before the synthesis, the analysis input before the grid step, the
 * tendencies or the updated node states and their synthesis layout before the analysis or update
 * that writes them -- with all-ones words (NaN in FP64 and FP32) just before that launch.  A
 * kernel that reads a value of its own sweep before it is written, padding it does not clear, or
 * a value left from an earlier sweep then produces NaN instead of the step's result; with correct
 * kernels the states are bitwise those of on = 0.  Extra fill launches; cached graphs are dropped. */
int sdc_debug_poison(sdc_handle h, int on);

/* Sizes and device memory of a handle. */
int sdc_get_info(sdc_handle h, sdc_info* info);

/* Launch variants of the two Legendre kernels (the Legendre parts of the spectral transforms of
 * Section 3.2).  Every variant computes the same sums in the same order from the same table
 * values (streamed or regenerated), so results are bitwise identical; only the speed differs
 * with truncation, batch and precision.
 *   syn_lat_tiles, syn_depth: 16-latitude tiles per synthesis workgroup and operand stages in
 *     flight per wave; the built pairs are (1, 8), (1, 4), (2, 4), (2, 2) (the default), (3, 2),
 *     (4, 2), (4, 1), (6, 1).
 *   ana_depth: table stages in flight per analysis wave, 2 (default) or 4.
 *   ana_interleave: 1 (default) runs the 4-state groups of one analysis task back to back on one
 *     XCD (shared table tile from its L2), 0 issues group after group. */
typedef struct {
    int syn_lat_tiles, syn_depth, ana_depth, ana_interleave;
    int fuse_update;   /* 1 (default): for M in {1, 2, 4} the node update of the next sweep runs in
                          the analysis kernel's epilogue, from tendencies that never leave its
                          workgroups (same arithmetic, bitwise the same states); 0: separate
                          update kernel.  Not changed by the autotuner. */
    int syn_recur;     /* 1: the synthesis regenerates Pbar_n^m and H_n^m in registers by the
                          upward three-term recurrence in n (Section 3.2 transforms; coefficients
                          and sectoral values precomputed at init, the same evaluation as the
                          stored tables, so the same results bit for bit) and reads only the
                          coefficient columns from HBM; 0: it reads the stored tables.  Built
                          for syn_lat_tiles 1, 2 and 4 (with their depths).  Chosen by the
                          autotuner with the synthesis shape. */
    int ana_recur;     /* 1: the analysis reads two stored Pbar values per latitude and four
                          rows and regenerates the table entries of those rows by the same
                          recurrence (a quarter of the table bytes; the same results bit for
                          bit); 0: it streams the tables.  Chosen by the autotuner. */
    int node_launch;   /* 0 (default): the f_E evaluations of the M nodes of a sweep (Algorithm 2's
                          parallel loop over m, Section 4.2) are one launch per kernel class; 1: one
                          launch set per node, one node after another, after a separate node-update
                          kernel -- the sequential counterpart of the time-parallel loop, bitwise
                          the same states, for measuring the speedup of evaluating the nodes
                          together (Section 4.7).  Handles of one member only (SDC_EINVAL
                          otherwise).  Applies to sdc_step, sdc_step_graph, sdc_step_taped and the
                          recomputation of sdc_step_adjoint.  Not changed by the autotuner. */
} sdc_plan;

/* The handle's current variants (of the launches over the node states of a sweep). */
int sdc_get_plan(sdc_handle h, sdc_plan* plan);

/* Select variants for every launch; SDC_EINVAL for a combination that is not built (the handle
 * keeps its plan).  fuse_update, syn_recur, ana_recur and node_launch must be 0 or 1.  Graphs
 * cached by sdc_step_graph are dropped and recaptured on their next call. */
int sdc_set_plan(sdc_handle h, const sdc_plan* plan);

/* Variants per launch shape.  A handle with M > 1 keeps two Legendre plans: one for the launches
 * over states = M states per member (the node states of a sweep, Algorithm 2's batched loop over
 * m) and one for the launches over states = 1 state per member (a step's first f_E, eval_explicit,
 * the f_E of the comparison integrators, the adjoint's first stage), which read the Legendre
 * tables for a quarter of the states and may prefer the variants that regenerate them.  All
 * variants give bitwise the same results.  fuse_update and node_launch belong to the step: set by
 * either call, reported by both.  states must be 1 or the configured M (SDC_EINVAL otherwise);
 * with M = 1 both name the same plan.  sdc_autotune chooses both plans. */
int sdc_get_plan_for(sdc_handle h, int states, sdc_plan* plan);
int sdc_set_plan_for(sdc_handle h, int states, const sdc_plan* plan);

/* Autotuner: times every built synthesis variant and every analysis variant on the handle's
 * stream, at both launch shapes of a step (batch x M states, and batch states with the synthesis
 * reading the states in place), reps launches each after one warm-up (1 <= reps <= 1000), and
 * switches each kernel of each shape to its fastest variant when that is at least 5 % faster
 * than the current one (the plan of the M-state launches is written to *chosen unless NULL; see
 * sdc_get_plan_for for the other).  Blocks
 * until the timing is done.  Overwrites the handle's synthesis and analysis workspaces (states
 * passed to other calls are not touched) and drops cached step graphs.  SDC_EHIP if a launch
 * fails (the previous plan is kept). */
int sdc_autotune(sdc_handle h, int reps, sdc_plan* chosen);

/* Copies of setup results to HOST buffers (blocking; for checking the FP64 setup):
 * mu[nlat], w[nlat] Gauss nodes and weights; tau[M], Q[M*M] (row-major) for 1 <= M <= cfg.M;
 * Pbar[(T-m+1)*(nlat/2)] and H[...] rows n = m..T over the northern latitudes j < nlat/2. */
int sdc_copy_grid(sdc_handle h, double* mu, double* w);
int sdc_copy_coefficients(sdc_handle h, int M, double* tau, double* Q);
int sdc_copy_legendre(sdc_handle h, int m, double* Pbar, double* H);

/* Ensembles of different truncations (one handle per truncation, each with its own members):
 * sdc_group_step advances every member of every handle by one dSDC step (Algorithm 2) as ONE graph
 * launch on the group's stream.  states[i] and dts[i] belong to members[i]; M and K are common
 * (<= every handle's configured M, K).  The graph is captured on the first call and whenever
 * states, dts, M or K change.  The member handles must outlive the group and must not be used on
 * other streams while a group step is in flight.  sdc_group_sync waits for the group's stream and
 * returns the first deferred error of a member.  sdc_group_create reserves a small device buffer
 * for the merged launches' arguments (released by sdc_group_free).
 * Modes (sdc_group_set_mode / sdc_group_get_mode):
 *   1: every phase of the step (each sweep's synthesis, grid step, analysis with its fused node
 *      update, or separate update) is ONE kernel launch over all members of all truncations --
 *      the batched loop over nodes of Algorithm 2 (Section 4.2) extended over the ensemble: each
 *      handle's workgroups form one range of the launch, with the Legendre variants of the handle
 *      with the most work (every variant gives the same results).  Needs members of one precision,
 *      the paper's split, one node per launch off, the same kind of node update (fused or not)
 *      and nlon in {96, 192, 384, 768}; sdc_group_step returns SDC_EUNSUPPORTED otherwise.
 *   0: each handle's own launches as a parallel branch of the graph.
 * A new group starts in mode 1 when its members allow it, else in mode 0.  Both modes give
 * bitwise the same states. */
typedef struct sdc_group_s* sdc_group;
int sdc_group_create(const sdc_handle* members, int n, void* hip_stream, sdc_group* out);
int sdc_group_step(sdc_group g, double* const* states, const double* dts, int M, int K);
int sdc_group_set_mode(sdc_group g, int mode);
int sdc_group_get_mode(sdc_group g, int* mode);

/* Group autotuner: when the members can share launches, times every built Legendre variant as a
 * merged launch at the node and one-state shapes (reps launches each) and keeps the fastest for
 * mode 1, then times reps whole steps of the given states in mode 1 and in mode 0 and keeps the
 * faster mode (*mode receives it unless NULL); otherwise selects mode 0.  The states are restored
 * afterwards (a device copy of each is allocated for the duration of the call); the members'
 * workspaces are overwritten.  Blocks until done.  Same argument rules as sdc_group_step. */
int sdc_group_autotune(sdc_group g, double* const* states, const double* dts, int M, int K, int reps,
                       int* mode);
int sdc_group_sync(sdc_group g);
int sdc_group_free(sdc_group g);

/* Message of the last error on the calling host thread ("" if none). */
const char* sdc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SDC_MI355X_H */
