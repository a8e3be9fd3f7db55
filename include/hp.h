/*
 * hp.h -- C ABI of the MI355X (gfx950) pressure-solve library libhp.so.
 *
 * The library solves the per-timestep implicit pressure equation of the semi-implicit low-Mach
 * scheme (paper, Section 2: eq. Poiss with the coefficients of eqs. cpoiss and kappapoiss,
 * homogeneous Neumann boundary condition eq. vonNeumannBC, periodic horizontal boundaries as in
 * Section 5), multiplied through by dt^2:
 *
 *     (1 / (rho c^2)) p - dt^2 div((1/rho) grad p) = rhs            (rhs = dt^2 f)
 *
 * on a cell-centred equidistant box. Discretely, with m_a = 1/(rho_a c2_a) and, for every face f
 * between adjacent cells a and b along axis d, w_f = dt^2 * (2 / (rho_a + rho_b)) / h_d^2 (the
 * face factor of the face-velocity update, step (viii) of the fractional-step algorithm):
 *
 *     (A p)_a = m_a p_a + sum_{f at a} w_f (p_a - p_b).
 *
 * A periodic axis with n >= 2 has a wrap face between cells 0 and n-1 (two faces when n = 2);
 * a Neumann boundary face carries no flux; an axis with n = 1 has no faces. A is symmetric
 * positive definite when rho, c2 > 0 (the Lax-Milgram conditions of Section 2).
 *
 * Layout of every cell array: FP64 (or FP32 where stated), nx*ny*nz entries,
 * index = i + nx*(j + ny*k), x fastest. Pointers named "device" are HIP device pointers on the
 * device that was current at hp_setup; the caller owns them. All work is ordered on the
 * handle's stream (default: the null stream; see hp_set_stream).
 *
 * Errors: every int-returning call returns HP_OK (0) or a negative code below; a message is kept
 * per thread (hp_last_error). A handle is not thread-safe; separate handles are independent.
 */
#ifndef HP_H
#define HP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hp_handle hp_handle;

/* Grid: cells per axis and spacings (x, y, z). ny = 1 (or nx = 1) gives a 2D problem. */
typedef struct {
    int nx, ny, nz;
    double hx, hy, hz;
} hp_grid;

/* Boundary kind per axis: HP_BC_PERIODIC or HP_BC_NEUMANN (homogeneous, eq. vonNeumannBC). */
enum { HP_BC_PERIODIC = 0, HP_BC_NEUMANN = 1 };
typedef struct {
    int x, y, z;
} hp_bc;

/* Return codes. */
enum {
    HP_OK = 0,
    HP_EINVAL = -1,      /* null pointer, n < 1, h <= 0, dt <= 0, tol <= 0, odd periodic n > 1,
                            bad option key or value, level out of range */
    HP_EDOMAIN = -2,     /* rho or c2 <= 0 or not finite (Lax-Milgram conditions violated) */
    HP_ENOMEM = -3,      /* device or host allocation failed */
    HP_EHIP = -4,        /* HIP runtime error (message kept) */
    HP_ENAN = -5,        /* non-finite right-hand side or iterate */
    HP_ENOCONV = -6,     /* iteration cap reached; p holds the last iterate, stats are filled */
    HP_EBREAKDOWN = -7,  /* p^T A p <= 0 in CG (cannot happen for valid SPD input) */
    HP_EIO = -8          /* a checkpoint file cannot be opened, read or written, or is not one */
};

/* Solver modes (HP_OPT_MODE). */
enum {
    HP_MODE_JACOBI_PCG = 0,  /* FP64 CG with diagonal preconditioner */
    HP_MODE_FP64_MGPCG = 1,  /* FP64 CG preconditioned by one geometric-multigrid V-cycle */
    HP_MODE_MIXED_IR = 2,    /* FP64 iterative refinement around an FP32 MG-PCG inner solve */
    HP_MODE_LEARNED = 3      /* FP64 flexible CG, preconditioner = network then V-cycle (needs
                                hp_attach_net); stops on the same FP64 true residual */
};

/* Option keys for hp_set_option / hp_get_option. */
enum {
    HP_OPT_MODE = 1,          /* one of HP_MODE_*; default HP_MODE_FP64_MGPCG */
    HP_OPT_MAX_ITER = 2,      /* CG iteration cap (total inner iterations in MIXED_IR); 1000 */
    HP_OPT_NU_PRE = 3,        /* red-black Gauss-Seidel pre-smoothing sweeps, 1..8; default 1 */
    HP_OPT_NU_POST = 4,       /* post-smoothing sweeps, 1..8; default 1 */
    HP_OPT_INNER_TOL = 5,     /* MIXED_IR: relative residual reduction per inner solve; 1e-5 */
    HP_OPT_MAX_OUTER = 6,     /* MIXED_IR: refinement-step cap; default 20 */
    HP_OPT_COARSEST_MAX = 7,  /* read-only after setup: max cells of the coarsest level (512) */
    HP_OPT_LAYOUT = 8         /* finest-level storage inside the handle: 1 = red-black split (each
                                 x row stores its red cells, then its black cells; the default
                                 where the grid allows it: nx even, nx >= 64, ny >= 4, nz >= 8
                                 and every axis coarsened at least once), 0 = natural order.
                                 Vectors passed through this API are always in natural order;
                                 setting 1 where the grid does not allow it is HP_EINVAL */,
    HP_OPT_KERNEL_TIMING = 9, /* 1: time finest-level kernels inside FP64 solves (hp_stats); 0 */
    HP_OPT_FACE_RULE = 10     /* value of kappa = 1/rho on a face between cells a and b (Section 2,
                                 eq. kappapoiss; the paper leaves it to the discretisation):
                                 0 (default) 2 / (rho_a + rho_b), the factor of the face-velocity
                                 update of step (viii); 1 (1/rho_a + 1/rho_b) / 2, the mean of the
                                 two cells' kappa. Applies to every level, the smoother and the
                                 coarsest solve; may be changed between solves (recomputes the
                                 rule-dependent setup, no allocation) */
};

/* Statistics of the last hp_solve. */
typedef struct {
    int iterations;        /* CG iterations (all inner iterations in MIXED_IR) */
    int outer_iterations;  /* MIXED_IR refinement steps (0 otherwise) */
    int converged;         /* 1 if the true relative residual met tol */
    int restarts;          /* CG restarts from the true residual */
    double rel_residual;   /* final true ||rhs - A p||_2 / ||rhs||_2, computed in FP64 */
    double time_ms;        /* wall time of hp_solve on the stream (HIP events) */
    int levels;            /* multigrid levels */
    int status;            /* return code of the solve */
    int fallback;          /* MIXED_IR: 1 if refinement stagnated and FP64 MG-PCG finished */
    /* with HP_OPT_KERNEL_TIMING on (FP64 solves): finest-level launches timed with HIP events on
       the handle's stream during the solve (attached to the dispatches; split layout only), and
       their average duration */
    int timed_sweeps;      /* red-black half sweeps (both post-smoothing sweeps) */
    double sweep_ms;
    int timed_applies;     /* operator applies q = A p of the CG iteration */
    double apply_ms;
} hp_stats;

/*
 * Build a solver for the operator A on `grid` with boundary kinds `bc`.
 *   rho, c2  device FP64 cell arrays (density and squared sound speed); copied, so the caller may
 *            reuse them on return.
 *   dt       time step (> 0).
 * Validates sizes (n >= 1, h > 0, periodic n even or 1), rho, c2 > 0 and finite. Allocates all
 * device workspace (hp_solve allocates nothing), builds the multigrid hierarchy, and assembles
 * and inverts the coarsest operator in FP64 on the device. On success *out receives the handle.
 */
int hp_setup(const hp_grid* grid, const double* rho, const double* c2, double dt,
             const hp_bc* bc, hp_handle** out);

/*
 * Solve A p = rhs to the true relative residual ||rhs - A p||_2 <= tol ||rhs||_2.
 *   rhs  device FP64, read only (the scaled right-hand side dt^2 f of eq. Poiss)
 *   p    device FP64, in: initial guess (zeros, or the previous pressure as a warm start),
 *        out: solution. rhs == 0 gives p = 0.
 * Synchronises the handle's stream before returning (convergence is decided on the host).
 * Returns HP_OK, HP_ENOCONV (p holds the last iterate), HP_ENAN, HP_EBREAKDOWN or HP_EHIP.
 */
int hp_solve(hp_handle* h, const double* rhs, double* p, double tol);

/* Release everything owned by the handle. NULL-safe. */
void hp_free(hp_handle* h);

/* Use `stream` (a hipStream_t) for all later work of this handle. */
int hp_set_stream(hp_handle* h, void* stream);

int hp_set_option(hp_handle* h, int key, double value);
int hp_get_option(const hp_handle* h, int key, double* value);

/*
 * Replace rho, c2 and dt (same grid): re-derives every level and the coarsest inverse without
 * reallocating. Same validation as hp_setup.
 */
int hp_update_coefficients(hp_handle* h, const double* rho, const double* c2, double dt);

/*
 * The operator with the two densities of eqs. cpoiss and kappapoiss (Section 2): the mass term
 * takes the density of time level n and the face coefficient that of time level n+1,
 *
 *     m_a = 1 / (rho_n_a c2_a),   w_f = dt^2 * (2 / (rho_np1_a + rho_np1_b)) / h_d^2.
 *
 *   rho_n, rho_np1, c2  device FP64 cell arrays (natural layout), copied; all must be positive
 *                       and finite (HP_EDOMAIN otherwise).
 * Everything else is as hp_setup / hp_update_coefficients (which are these calls with
 * rho_np1 = rho_n). The learned stage then sees log rho_np1 and -log(rho_np1 m) as its
 * coefficient channels.
 */
int hp_setup_two_density(const hp_grid* grid, const double* rho_n, const double* rho_np1,
                         const double* c2, double dt, const hp_bc* bc, hp_handle** out);
int hp_update_coefficients_two_density(hp_handle* h, const double* rho_n, const double* rho_np1,
                                       const double* c2, double dt);

/*
 * Inhomogeneous Neumann data (the stability problem of Section 2 prescribes the outward normal
 * derivative of the solution on the boundary): adds the known boundary flux to the right-hand
 * side of the cells next to boundary `side` (0: low, 1: high) of `axis` (0 x, 1 y, 2 z), which
 * must be a Neumann axis of the handle (the operator itself keeps no flux there):
 *
 *     rhs_a += dt^2 q_f / h_axis
 *
 *   q    device FP64, one value per boundary face: the prescribed outward normal flux
 *        kappa dphi/dn (with kappa = 1, as in the stability problem, the normal derivative; a
 *        caller with derivative data g and face coefficient kappa passes kappa g), indexed over the
 *        plane of the two other axes with the lower-numbered axis fastest
 *        (axis x: j + ny k; axis y: i + nx k; axis z: i + nx j); read only.
 *   rhs  device FP64 cell array (natural layout), updated in place; stream-ordered, no sync.
 * Errors: HP_EINVAL (null pointer, axis or side out of range, axis not Neumann), HP_EHIP.
 */
int hp_neumann_rhs(hp_handle* h, int axis, int side, const double* q, double* rhs);

int hp_get_stats(const hp_handle* h, hp_stats* out);

/* Thread-local message of the last error ("" if none). */
const char* hp_last_error(void);

/* ---- The steps either side of the solve (Section 2, "The Algorithm") ---------------------------
 * Natural-layout FP64 cell arrays of the handle's grid (nx*ny*nz entries each, device pointers,
 * caller-owned). A momentum argument is three consecutive cell arrays: the x, y and z components.
 * Boundaries are the handle's: periodic axes wrap; at a closed (Neumann) boundary the interface
 * velocity is zero and the interface pressure is the adjacent cell's (eq. vonNeumannBC); an axis
 * of one cell has no gradient or divergence. dt is the handle's. Stream-ordered, no sync.
 */

/* Fields that form the right-hand side. */
typedef struct {
    const double* rho_n;     /* density at time n */
    const double* c2_n;      /* squared sound speed at time n */
    const double* p_n;       /* pressure at time n */
    const double* mom_n;     /* (rho u)^n, 3 cell arrays */
    const double* rho_np1;   /* density at time n+1 (after the explicit step) */
    const double* mom_star;  /* (rho u)* after the explicit step, 3 cell arrays */
    const double* visc;      /* NULL, or per cell the group u.div(tau) - div(u.tau) + div(K grad T) at time
                                n (viscous stress and heat conduction of the explicit part) */
    const double* temp_n;    /* NULL for one component (eq. fpoiss); for two (eq. fpoiss2) the
                                temperature T^n, with conc_n, rkc_n and r_gas: */
    const double* conc_n;    /* mass fraction c^n */
    const double* rkc_n;     /* rho^n kappa_c per cell (interface value: mean of the two cells) */
    double r_gas;            /* gas constant R_gas */
} hp_rhs_fields;

/*
 * Steps (iv)-(v): the right-hand side of the pressure equation, b = dt^2 f with f of eq. fpoiss
 * (eq. fpoiss2 when temp_n is given), in the scaling of hp_solve:
 *
 *   b = m (P^n - dt u^n . grad P^n) - dt div u* - (2 dt / 3)(m / rho^n) G
 *       - (3 dt / 4) m R_gas T^n div(rho^n kappa_c grad c^n),     m = 1 / (rho^n c2^n),
 *
 * u^n = (rho u)^n / rho^n; grad P^n from the interface pressure of eq. pbnd (weights rho^n) and the
 * central difference of eq. nablaP; div u* from the interface velocities of eq. step1 applied to
 * (rho u)* and rho^{n+1}. rhs must not alias an input. Errors: HP_EINVAL (null handle, fields,
 * rhs or required field), HP_EHIP.
 */
int hp_pressure_rhs(hp_handle* h, const hp_rhs_fields* f, double* rhs);

/* Fields of the update after the solve. */
typedef struct {
    const double* p;         /* predicted pressure P^{n+1} (the solution of hp_solve) */
    const double* rho_np1;   /* density at time n+1 */
    const double* mom_star;  /* (rho u)*, 3 cell arrays */
    const double* e_star;    /* total energy e* after the explicit step */
    double* mom_out;         /* out: (rho u)^{n+1}, 3 cell arrays */
    double* uface_out;       /* out: interface velocities u^{n+1} on the high side of every cell
                                along x, y, z (3 cell arrays; 0 at a closed high end) */
    double* e_out;           /* out: total energy e^{n+1} */
} hp_update_fields;

/*
 * Steps (vii)-(ix): momentum (rho u)^{n+1} = (rho u)* - dt grad P (eqs. momupdate, pbnd and
 * nablaP with rho^{n+1}); interface velocities u^{n+1}_{i+1/2} = u*_{i+1/2}
 * - dt (P_{i+1} - P_i) / h * 2 / (rho^{n+1}_{i+1} + rho^{n+1}_i) (step (viii), u* by eq. step1);
 * energy e^{n+1} = e* - dt (P div u^{n+1} + u^{n+1} . grad P) (eq. enupdate, div from the new
 * interface velocities, u^{n+1} = (rho u)^{n+1} / rho^{n+1}). Outputs must not alias inputs or each
 * other. Errors: HP_EINVAL (null pointer, aliasing), HP_EHIP.
 */
int hp_pressure_update(hp_handle* h, const hp_update_fields* f);

/*
 * Steps (i)-(iii) for inviscid flow, the explicit part of a time step: interface velocities of
 * eq. step1; the modified advective flux q_face u_{i+1/2} of each conserved field (rho, the three
 * momenta, e), with q_face reconstructed componentwise on the upwind side of the interface by
 * second-order ENO (the smaller in magnitude of the two one-sided differences; the advective
 * Jacobian has all eigenvalues u, so no characteristic projection is needed); and
 * q* = q - dt div(flux) with the handle's dt, giving rho^{n+1}, (rho u)* and e*. Closed boundaries
 * carry no flux and mirror the edge cell for the reconstruction; periodic axes wrap.
 *   rho, e   cell arrays; mom: 3 cell arrays (x, y, z). Outputs likewise; no output may alias an
 *            input or another output. Errors: HP_EINVAL, HP_EHIP.
 */
int hp_advect(hp_handle* h, const double* rho, const double* mom, const double* e, double* rho_out,
              double* mom_out, double* e_out);

/*
 * Step (x), ideal gas: P = (gamma - 1)(e - |rho u|^2 / (2 rho)) and, if c2 is not NULL,
 * c2 = gamma P / rho (the squared sound speed of eq. cpoiss). Cell arrays (mom: 3 arrays) of the
 * handle's grid; gamma > 1. Errors: HP_EINVAL, HP_EHIP.
 */
int hp_eos_ideal(hp_handle* h, const double* rho, const double* mom, const double* e, double gamma,
                 double* p, double* c2);

/* y = a x + b y for device vectors of n entries (the Runge-Kutta averages of a time step), on the
 * handle's stream. Errors: HP_EINVAL (null vector with n > 0, n < 0), HP_EHIP. */
int hp_axpby(hp_handle* h, double a, const double* x, double b, double* y, long long n);

/* ---- Building blocks of the solve, exposed for verification and composition ------------------
 * Levels are numbered 0 (fine) .. hp_num_levels()-1 (coarsest). Vectors of level l are device
 * arrays of that level's cell count; FP32 variants ("_f32") act on the FP32 copies of the
 * coefficients used by the mixed-precision inner solve.
 */

int hp_num_levels(const hp_handle* h);

/* Cells per axis (n[3]) and spacings (hs[3]) of level l; either pointer may be NULL. */
int hp_level_info(const hp_handle* h, int level, int* n, double* hs);

/* y = A_l x (flux form) on level l. */
int hp_apply(hp_handle* h, int level, const double* x, double* y);
int hp_apply_f32(hp_handle* h, int level, const float* x, float* y);

/*
 * One red-black Gauss-Seidel half sweep of colour `colour` (0 = red: (i+j+k) even) on level l:
 * for every cell a of that colour z_a <- (r_a + sum_f w_f z_b) / (m_a + sum_f w_f).
 * Cells of the other colour are left unchanged.
 */
int hp_smooth(hp_handle* h, int level, const double* r, double* z, int colour);
int hp_smooth_f32(hp_handle* h, int level, const float* r, float* z, int colour);

/*
 * Residual restriction to level l+1: rc = R (r - A_l z), R = P^T / 2 per coarsened axis
 * ((1,3,3,1)/8 interior weights; Neumann ends mirrored, periodic ends wrapped).
 */
int hp_restrict_residual(hp_handle* h, int level, const double* r, const double* z, double* rc);
int hp_restrict_residual_f32(hp_handle* h, int level, const float* r, const float* z, float* rc);

/* Trilinear prolongation and correction from level l+1: z += P ec (weights 3/4, 1/4 per axis). */
int hp_prolong_add(hp_handle* h, int level, const double* ec, double* z);
int hp_prolong_add_f32(hp_handle* h, int level, const float* ec, float* z);

/* Coarsest-level solve x = A_c^-1 b in FP64 (FP32 variant converts in and out). */
int hp_coarse_solve(hp_handle* h, const double* b, double* x);
int hp_coarse_solve_f32(hp_handle* h, const float* b, float* x);

/* One multigrid V-cycle z = M r on the fine level (the preconditioner of FP64_MGPCG). */
int hp_precond(hp_handle* h, const double* r, double* z);
int hp_precond_f32(hp_handle* h, const float* r, float* z);

/*
 * r = rhs - A p on the fine level in FP64; if rel is not NULL it receives
 * ||r||_2 / ||rhs||_2 (synchronises the stream).
 */
int hp_residual(hp_handle* h, const double* rhs, const double* p, double* r, double* rel);

/* Deterministic FP64 dot product of device vectors of n entries (synchronises the stream); x and
 * y may be NULL when n = 0 (the result is 0). Lengths whose first reduction stage needs more
 * partial sums than the handle holds (it holds those of a vector of the fine grid's size) are
 * HP_EINVAL. */
int hp_dot(hp_handle* h, const double* x, const double* y, long long n, double* out);

/*
 * For callers that cannot allocate (code under stream capture, tight serving loops): the same
 * deterministic dot product as hp_dot, bitwise, with no handle and no allocation of any kind.
 *   x, y     device FP64 vectors of n entries (may be NULL when n = 0); read only.
 *   n        >= 0. The first reduction stage writes one partial sum per workgroup (at most 2048,
 *            one per 1024 entries, for any n) into a 16 KiB static device array of the library,
 *            one per GPU, held until the process ends; lengths needing more are HP_EINVAL.
 *   result   device pointer to one FP64 value (caller-owned) that receives <x, y>.
 *   stream   hipStream_t the two kernels are enqueued on (NULL: the null stream); the call
 *            returns without synchronising.
 * Every call on a GPU uses that GPU's one static array: calls that overlap on one GPU (on
 * different streams or host threads without ordering between them) race and may return wrong
 * sums. Errors: HP_EINVAL (null result, null x or y with n > 0, n < 0), HP_EHIP; the message is
 * in hp_noalloc_last_error().
 */
int hp_dot_noalloc(const double* x, const double* y, long long n, double* result, void* stream);
const char* hp_noalloc_last_error(void);

/*
 * dst = src for n doubles with 16-byte non-temporal loads and stores: the plain streaming pass
 * against which the benchmark states measured bandwidth (it is no step of the solve). Device
 * pointers, 16-byte aligned, not overlapping; enqueued on `stream` (a hipStream_t, NULL: the null
 * stream) without synchronising. Errors: HP_EINVAL (null pointer with n > 0, n < 0, misaligned
 * or overlapping buffers), HP_EHIP.
 */
int hp_stream_copy(const double* src, double* dst, long long n, void* stream);

/* ---- Learned warm start / preconditioner -------------------------------------------------
 * A small 3D U-Net (levels n, n/2, n/4 with 16/32/64 channels, 3x3x3 convolutions padded
 * periodically in x, y and with zeros in z, 2x2x2 mean pooling, nearest upsampling, skip
 * concatenations, ReLU, 1x1x1 output head) in bfloat16 on the matrix cores with FP32
 * accumulation. Its input per cell is (b/s, log rho, log c2, p_prev/s) with s = RMS(b); its
 * output y gives the estimate x = s * out_scale * y of the solution of A x = b. Not part of the
 * paper's method: it stands beside the multigrid solver, which decides accuracy.
 *
 * Parameters: one flat FP32 device vector of hp_nn_num_params() entries; per convolution
 * W[o][t][c] (c fastest) then bias[o], in the order in->16, 16->16, 16->32, 32->32, 32->64,
 * 64->64, 96->32, 32->32, 48->16, 16->16 (taps t = (dz+1)*9 + (dy+1)*3 + (dx+1)); then the head
 * weights [16] and bias. Activations are channels-last ([cell][channel]).
 */
typedef struct hp_net hp_net;

long long hp_nn_num_params(void);

/* Network workspace for an nx x ny x nz grid (each a multiple of 4, fewer than 2^31 cells in
 * all, else HP_EINVAL); training != 0 also allocates gradients and Adam state. Parameters start
 * at zero. */
int hp_nn_create(int nx, int ny, int nz, int training, hp_net** out);
void hp_nn_free(hp_net* net);
int hp_nn_set_stream(hp_net* net, void* stream);
const char* hp_nn_last_error(void);

/* Copy parameters in/out (device FP32, hp_nn_num_params() entries). */
int hp_nn_set_params(hp_net* net, const float* params);
int hp_nn_get_params(hp_net* net, float* params);
int hp_nn_get_grad(hp_net* net, float* grad);
int hp_nn_set_output_scale(hp_net* net, double out_scale);

/* Checkpoints: the parameters and the output scale in one binary file (little-endian: the 8
 * bytes "HPNET01\0", int64 parameter count, float64 output scale, the parameters as float32).
 * hp_nn_save writes the network's current ones (synchronises its stream); hp_nn_load replaces
 * them (any grid: the parameters do not depend on it) and leaves the network unchanged when it
 * rejects the file. HP_EIO for a file that cannot be opened, read or written, a wrong magic or a parameter
 * count other than hp_nn_num_params(); HP_EINVAL for null arguments. */
int hp_nn_save(hp_net* net, const char* path);
int hp_nn_load(hp_net* net, const char* path);

/* x = s * out_scale * net(b/s, log rho, log c2, p_prev/s); p_prev may be NULL (zeros).
 * All device FP64 cell arrays. */
int hp_nn_forward(hp_net* net, const double* b, const double* rho, const double* c2,
                  const double* p_prev, double* x);

/* One Adam step (lr) on the mean squared error between the network output and
 * x_target / (s * out_scale); *loss receives the loss before the step (synchronises). */
int hp_nn_train_step(hp_net* net, const double* b, const double* rho, const double* c2,
                     const double* p_prev, const double* x_target, float lr, double* loss);

/* Raw access for verification: input features [cell][8] bfloat16 (channels 4..7 zero) ->
 * y [cell] FP32; loss and parameter gradient of mean (y - target)^2 (hp_nn_get_grad);
 * Adam step with the current gradient. */
int hp_nn_forward_raw(hp_net* net, const unsigned short* in, float* y);
int hp_nn_loss_grad_raw(hp_net* net, const unsigned short* in, const float* target, double* loss);
int hp_nn_adam(hp_net* net, float lr);

/* One Adam step on the relative A-norm error of the network's estimate of the solution x of
 * A x = b (A of the handle; the net must be a training network on the same grid):
 * loss = <e, A e> / <x, A x>, e = s * out_scale * net(b, log rho, log c2, p_prev) - x.
 * *loss receives the loss before the step (synchronises). Allocates the learned stage's work
 * vectors on first use, as hp_attach_net does. */
int hp_nn_train_step_anorm(hp_handle* h, hp_net* net, const double* b, const double* p_prev,
                           const double* x, float lr, double* loss);

/* Use `net` (same grid as the handle; NULL detaches) in HP_MODE_LEARNED and hp_warm_start.
 * Allocates the learned stage's three work vectors of the fine grid on first use (shared with
 * hp_nn_train_step_anorm, whichever comes first). */
int hp_attach_net(hp_handle* h, hp_net* net);

/* Initial guess x = g y from the attached network, y = net(b, p_prev) (p_prev may be NULL), with
 * g = <b, y> / <y, A y> the step minimising the A-norm error of x (g = 0, i.e. x = 0, if the
 * network points uphill). Use before hp_solve; the solve's accuracy does not depend on it. */
int hp_warm_start(hp_handle* h, const double* b, const double* p_prev, double* x);

#ifdef __cplusplus
}
#endif

#endif /* HP_H */
