/*
 * lbm.h -- C ABI of the MI355X lock-exchange lattice Boltzmann library.
 *
 * Method: Adekanye et al., "GPU accelerated lattice Boltzmann method
 * simulations of dilute gravity currents" (arXiv 2112.08479). One time step
 * is the collide-then-stream update of Eq. 17 for the flow populations and
 * Eq. 28 for the scalar populations, coupled through the Boussinesq force of
 * Eq. 11, with half-way bounce-back walls (no slip, no flux) at x = 0, x = nx,
 * z = 0, z = nz and a periodic span y (Sec. 2.5).
 *
 *   model LBM_CUMULANT27_Q7    : D3Q27 cumulant collision (Eq. 36, 54-58)
 *                                and a D3Q7 BGK scalar (Eq. 28-30 on D3Q6 +
 *                                rest)
 *   model LBM_BGK19_SMAG_Q6    : D3Q19 BGK + Guo forcing (Eq. 21-26) with
 *                                Smagorinsky eddy viscosity (Eq. 32-35) and
 *                                a D3Q6 BGK scalar (Eq. 28-31)
 *   model LBM_CUMULANT27_FCM27 : the D3Q27 cumulant collision and a D3Q27
 *                                factorized-central-moment scalar (Eq. 37-51)
 *
 * Conventions shared by every entry point
 *   - Every function returns 0 (LBM_OK) or a negative LBM_E* code and never
 *     throws across the ABI; lbm_last_error() gives a thread-local message
 *     for the last failure on the calling thread.
 *   - Device memory is owned by the caller. lbm_create carves its buffers out
 *     of a caller workspace; the handle owns only host memory. All pointers
 *     named *_dev are device pointers, host_* are host pointers.
 *   - Work is queued on the caller's HIP stream in order. Only
 *     lbm_diagnostics, lbm_get_populations, lbm_set_populations,
 *     lbm_checkpoint_save, lbm_checkpoint_load and lbm_adjoint_run
 *     synchronise that stream.
 *   - Node (i, j, k) has linear index i + nx (j + ny k); x = i is the
 *     streamwise direction, y = j the span, z = k the vertical (gravity
 *     along -z, Eq. 10). Fields passed in or out (chi0, moments, gradients,
 *     wall stress) use that index. The population buffers inside the
 *     workspace are x-blocked: element (a, i, row = j + ny k) sits at
 *     (row ceil(nx/64) + i/64) (qt 64) + 64 a + i % 64; they are reached only
 *     through the calls below (checkpoints copy them whole).
 *   - Population order (for the get/set hooks): D3Q19 in the order printed
 *     in Eq. 23; D3Q27 = that list followed by the corners (1,1,1),
 *     (-1,-1,-1), (1,1,-1), (-1,-1,1), (1,-1,1), (-1,1,-1), (1,-1,-1),
 *     (-1,1,1); D3Q6 in the order of Eq. 31; D3Q7 = rest + D3Q6.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid argument or configuration */
  LBM_ENOMEM = -2,    /* workspace or slot too small */
  LBM_EDEVICE = -3,   /* a HIP runtime call failed */
  LBM_ENODEV = -4,    /* no GPU visible */
  LBM_EUNSTABLE = -5, /* the state holds non-finite values */
  LBM_ESTATE = -6     /* call out of order (e.g. step before init) */
};

/* Models (Sec. 2.3):
 *   LBM_CUMULANT27_Q7    D3Q27 cumulant fluid (Eq. 54-58) + D3Q7 BGK scalar
 *                        (Eq. 28-30);
 *   LBM_BGK19_SMAG_Q6    D3Q19 BGK fluid with Guo forcing and Smagorinsky
 *                        eddy viscosity (Eq. 21-26, 32-35) + D3Q6 BGK scalar
 *                        (Eq. 28-31);
 *   LBM_CUMULANT27_FCM27 D3Q27 cumulant fluid + D3Q27 factorized-central-
 *                        moment scalar (Eq. 36-51), the first-order moments
 *                        relaxed with omega_100 = 1/tau_phi (Eq. 51) and the
 *                        other non-conserved moments with rate 1.
 * The C_s > 0 eddy viscosity and its scalar diffusivity nu_T / Sc_T apply to
 * every model. */
enum { LBM_CUMULANT27_Q7 = 0, LBM_BGK19_SMAG_Q6 = 1, LBM_CUMULANT27_FCM27 = 2 };

/* Storage type of the populations. The flow populations are stored as
 * deviations f_q - w_q from the lattice rest state (the split of Eq. 52-53),
 * the scalar populations as raw values. Arithmetic is FP64 when the storage
 * is LBM_F64 and FP32 otherwise; global reductions are FP64. 16-bit stores
 * round to nearest even. LBM_BF16_F16S stores the flow in bfloat16 and the
 * scalar in IEEE half precision (the scalar's 0..1 range needs mantissa, not
 * exponent: bfloat16's 8-bit mantissa loses scalar mass). */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2, LBM_BF16 = 3, LBM_BF16_F16S = 4 };

/* Output element type for lbm_moments. */
enum { LBM_OUT_F32 = 1, LBM_OUT_F64 = 0 };

typedef struct {
  uint32_t struct_size;   /* must be sizeof(lbm_config) */
  int32_t nx, ny, nz;     /* nodes; depth H = nz lattice units */
  int32_t model;          /* LBM_CUMULANT27_Q7, LBM_BGK19_SMAG_Q6 or
                             LBM_CUMULANT27_FCM27 */
  int32_t storage;        /* LBM_F64 / LBM_F32 / LBM_F16 / LBM_BF16 /
                             LBM_BF16_F16S */
  double re_b;            /* buoyancy Reynolds number U_b H / nu0 (Eq. 12-14) */
  double sc;              /* Schmidt number nu0 / D0 */
  double g_prime;         /* reduced gravity, lattice units */
  double ub_lu;           /* > 0: U_b in lattice units, g' = ub_lu^2 / nz
                             (the paper's convention U_b = 0.03, Sec. 2.5) */
  double cs_smag;         /* Smagorinsky constant C_s; 0 disables the LES
                             (convention: smag_paper_form below) */
  double sc_t;            /* turbulent Schmidt number */
  double omega_bulk;      /* cumulant trace (bulk) relaxation rate, (0, 2) */
  double omega3, omega4, omega5, omega6; /* cumulant rates of order 3..6 */
  /* 1: the parametrised cumulant of the paper's VirtualFluids runs (Sec. 2.3;
   * the method of Geier, Pasquali and Schoenherr, J. Comput. Phys. 348,
   * 2017): the third-order rates are functions of omega1 = 1/tau0 and
   * omega_bulk chosen for fourth-order accurate shear diffusion
   * (lbm_params.w_plus, w_minus, w_111), the fourth-order cumulants relax
   * with rate 1 onto equilibria proportional to the velocity gradients
   * (coefficients coef_a, coef_b), orders 5 and 6 with rate 1 towards 0.
   * Needs a cumulant model, cs_smag = 0 (the method runs without a sub-grid
   * model), omega3..omega6 = 1 (they are replaced), omega1 != omega_bulk and
   * finite rates. 0: every cumulant of order n relaxes with omega_n. */
  int32_t parametrized;
  /* limiter lambda of the third-order relaxation in parametrised mode: each
   * rate w becomes w + (1 - w)|X| / (|X| + lambda) for its own third-order
   * quantity X (a cumulant of f / rho); 0 = no limiter; >= 0 */
  double limiter;
  /* 1: the Smagorinsky closure as printed in Eq. 32, nu_T = C_s Delta^2 |S|
   * (C_s to the first power; the paper's C_s = 0.03 equals the standard
   * form's 0.173); 0: the standard nu_T = (C_s Delta)^2 |S|. Delta = 1. */
  int32_t smag_paper_form;
} lbm_config;

/* Derived lattice-unit parameters (Sec. 2.5, Eq. 25, 30). */
typedef struct {
  double u_b;       /* sqrt(g' H) */
  double g_prime;
  double nu0;       /* U_b H / Re_b */
  double tau0;      /* 3 nu0 + 1/2 */
  double d0;        /* nu0 / Sc */
  double tau_phi0;  /* 1/2 + D0 / cs_phi^2 */
  double cs2_phi;   /* 1/4 (D3Q7) or 1/3 (D3Q6, D3Q27) */
  int32_t q_flow, q_scalar;
  /* parametrised cumulant (0 unless lbm_config.parametrized): rates of
   * C_120 + C_102 (and permutations), of C_120 - C_102 (and permutations)
   * and of C_111; fourth-order equilibrium coefficients A and B */
  double w_plus, w_minus, w_111, coef_a, coef_b;
} lbm_params;

/* Diagnostics of the state at the current step (pre-collision moments):
 *   mass = sum rho, chi_mass = sum chi (mass0 / chi_mass0: at initialisation);
 *   fw = sum over the bottom layer of nu0 (9 u_x(z=0) - u_x(z=1)) / 3
 *        (Eq. 62 with the half-way wall, Eq. 64), fw_nd = fw / (U_b^2 H^2);
 *   x_front: front position from the span-averaged concentration with
 *        threshold 0.02 (Sec. 3.1), linearly interpolated between node
 *        centres; x_f = x_front - x0 (gate position); x_f_nd = x_f / H;
 *   umax = max |u|; nonfinite = nodes whose rho, u or chi is not finite;
 *   t_nd = step U_b / H. */
typedef struct {
  int64_t step;
  double t_nd, mass, mass0, chi_mass, chi_mass0, fw, fw_nd;
  double x_front, x_f, x_f_nd, umax;
  int64_t nonfinite;
} lbm_diag;

typedef struct lbm_handle lbm_handle;

/* Host only. Fills *out from cfg (Sec. 2.5). LBM_EINVAL if cfg is invalid
 * (sizes < 1 or nx*ny*nz >= 2^31, unknown model/storage, Re_b, Sc, Sc_T <= 0,
 * g' < 0, tau0 <= 1/2, rates outside (0, 2), C_s < 0). */
int lbm_derive_params(const lbm_config* cfg, lbm_params* out);

/* Host only. Device workspace bytes lbm_create needs for cfg: two population
 * buffers (read / write) plus reduction scratch. 0 if cfg is invalid. */
size_t lbm_workspace_bytes(const lbm_config* cfg);

/* Host only. Bytes of one checkpoint slot: one population buffer and a
 * header (grid, model, storage, step counter, gate index, diagnostics at
 * initialisation). */
size_t lbm_state_bytes(const lbm_config* cfg);

/* Validates cfg (LBM_EINVAL, before any device work), checks for a GPU
 * (LBM_ENODEV) and the workspace size (LBM_ENOMEM), then builds a handle on
 * the current device. dev_workspace: caller-owned device memory of at least
 * lbm_workspace_bytes(cfg) bytes, 256-byte aligned, kept alive until
 * lbm_destroy. hip_stream: hipStream_t (NULL = default stream). */
int lbm_create(const lbm_config* cfg, void* dev_workspace, size_t bytes,
               void* hip_stream, lbm_handle** out);

/* Frees the handle (host memory only; never the caller's workspace). */
int lbm_destroy(lbm_handle* h);

/* Initial state of Sec. 2.5 at step 0: zero momentum (f = w), chi0 = 1 for
 * i < floor(lock_fraction nx), else 0, plus noise_amp (2U - 1) in the two
 * columns i = floor(lock_fraction nx) - 1 and floor(lock_fraction nx), with
 * U = (splitmix64(seed ^ (l * 0x9E3779B97F4A7C15)) >> 11) 2^-53 and l the
 * node's linear index; phi = w_phi chi0. Records mass0 and chi_mass0. */
int lbm_init_lock_exchange(lbm_handle* h, double lock_fraction, double noise_amp,
                           uint64_t seed);

/* Same with chi0 given as nx*ny*nz doubles in device memory (layout above);
 * lock_fraction only sets the gate position x0 used by the front diagnostic. */
int lbm_init_from_field(lbm_handle* h, const double* chi0_dev, double lock_fraction);

/* Queues n time steps (Eq. 17, 28). n = 0 is a no-op; n < 0 is LBM_EINVAL;
 * LBM_ESTATE before initialisation. Does not synchronise. */
int lbm_step(lbm_handle* h, int64_t n);

/* Pre-collision moments of the current state (Eq. 19-20, 27): rho, the
 * velocity u = (j + F/2)/rho, chi, nx*ny*nz elements each of type dtype
 * (LBM_OUT_F32 / LBM_OUT_F64) into caller device buffers; NULL skips one. */
int lbm_moments(lbm_handle* h, int dtype, void* rho_dev, void* ux_dev,
                void* uy_dev, void* uz_dev, void* chi_dev);

/* Bottom-wall shear stress of the current state in lattice units (Eq. 62,
 * mu = rho_bar nu0 with rho_bar = 1, Eq. 52): the second-order one-sided
 * slope through the two nearest fluid nodes (Sec. 3.2), which with the
 * half-way wall at distance 1/2 is tau_w(x, y) = nu0 (9 u_x(z=0) - u_x(z=1))/3,
 * u_x the signed streamwise velocity. tau_dev: nx*ny elements (index
 * y*nx + x); tau_bar_dev: nx elements, the span average of Sec. 3.2 (the
 * integrand of Eq. 66). Elements of type dtype (LBM_OUT_F32 / LBM_OUT_F64) in
 * caller device buffers; NULL skips one. Summed over the wall, tau_w is the
 * F_w of lbm_diag (Eq. 64). Needs nz >= 2 (LBM_EINVAL otherwise). Does not
 * synchronise. */
int lbm_wall_shear(lbm_handle* h, int dtype, void* tau_dev, void* tau_bar_dev);

/* Computes the diagnostics (FP64 reductions on the GPU), synchronises and
 * writes *out. Returns LBM_EUNSTABLE (with *out filled) if nonfinite > 0. */
int lbm_diagnostics(lbm_handle* h, lbm_diag* out);

/* Step counter of the handle. */
int lbm_get_step(const lbm_handle* h, int64_t* step);

/* Copies the population buffer and the header (grid, model, storage, step
 * counter, gate index x0, the diagnostics recorded at initialisation) into a
 * caller device slot of lbm_state_bytes(cfg) bytes; synchronises. */
int lbm_checkpoint_save(lbm_handle* h, void* dev_slot);
/* Restores a slot written by lbm_checkpoint_save into this handle, which may
 * be a fresh one (never initialised): the populations, the step counter, the
 * gate index and the initial diagnostics (mass0, chi_mass0), so that later
 * diagnostics match those of the saved run. LBM_EINVAL, with the handle left
 * unchanged, if the slot's header is not a checkpoint's or its grid, model or
 * storage differ from the handle's (the physics parameters may differ: a run
 * may be continued with another C_s, say). Synchronises. */
int lbm_checkpoint_load(lbm_handle* h, const void* dev_slot);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the diagnostics
 * of lbm_diagnostics for the state held in a checkpoint slot written by
 * lbm_checkpoint_save, without a handle or a workspace. cfg must have the
 * slot's grid, model and storage (LBM_EINVAL otherwise, or if the slot holds
 * no checkpoint header); its physics parameters (nu0 for F_w, U_b for the
 * non-dimensional values) are used as given. step, x_f and mass0/chi_mass0
 * come from the slot's header. The scratch of the diagnostics kernels (span
 * sums of chi, per-block partial sums, a result slot) is a static device
 * array of 32 MiB per GPU, held until the process ends: LBM_ENOMEM if the
 * grid needs more (nx * nz above about 4.1 million). Nothing is allocated.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other host threads, other streams) race and must be serialised by the
 * caller. hip_stream: the stream to run on (NULL = default); synchronises
 * it. Returns LBM_EUNSTABLE (with *out filled) if nonfinite > 0. */
int lbm_checkpoint_diagnostics(const lbm_config* cfg, const void* dev_slot, void* hip_stream,
                               lbm_diag* out);

/* Test hooks. Pre-collision populations at the current step as full values
 * (f, not f - w), float64, host arrays of q_flow*N and q_scalar*N in the
 * population order above. Synchronous. */
int lbm_get_populations(lbm_handle* h, double* host_f, double* host_phi);
int lbm_set_populations(lbm_handle* h, const double* host_f, const double* host_phi);

/* ------------------------------------------------------------------------
 * Differentiation form. J = w_front x_f(n) + w_fw (1/n) sum_{m=1..n} F_w(m)
 * (lattice units; x_f and F_w as in lbm_diag: front of Sec. 3.1, wall
 * friction of Eq. 62, 64) for an n-step run started from the current state,
 * which must be a fresh initialisation (step 0). The forward pass keeps a
 * checkpoint every k_ckpt steps; the reverse pass recomputes each segment and
 * runs the hand-written adjoint of the gather with bounce-back and of the
 * local collision (Eq. 17, 21-35, 37-51, 54-58; Sec. 2.3 for the
 * parametrised cumulant). Outputs: *J_out, *dJ_dcs (C_s),
 * *dJ_dsct (Sc_T) as host doubles and dJ/dchi0 (nx*ny*nz doubles, device;
 * chi0 enters through phi(0) = w_phi chi0). Non-smooth points: zero
 * subgradient of sqrt(Q) at Q = 0; the front uses the active column i* and
 * the first depth maximum. The cumulant models need omega3..omega6 = 1 or
 * the parametrised mode (its limiter differentiated as
 * d/dX [X (1 - w)(1 - |X|/(|X| + lambda))] = (1 - w)(1 - q)^2,
 * q = |X|/(|X| + lambda)); storage LBM_F32 or LBM_F64 (LBM_EINVAL
 * otherwise); LBM_ESTATE if the
 * handle is not at step 0. adj_ws: device scratch of
 * lbm_adjoint_workspace_bytes(cfg, n, k_ckpt) bytes (LBM_ENOMEM if smaller).
 * When one population buffer is at most 64 MiB (a cache-resident grid whose
 * kernels are latency bound) and there are two segments or more, the
 * workspace holds two trajectory sets and the run recomputes segment s - 1 on
 * a second stream of its own (non-blocking, default priority, made on the
 * first such run and released by lbm_destroy) while segment s is reversed on
 * the handle's stream; events order the two, and the second stream is idle
 * when the call returns. Leaves the handle at step n. Synchronises. */
size_t lbm_adjoint_workspace_bytes(const lbm_config* cfg, int64_t n_steps, int64_t k_ckpt);
int lbm_adjoint_run(lbm_handle* h, int64_t n_steps, int64_t k_ckpt, double w_front,
                    double w_fw, void* adj_ws, size_t adj_bytes, double* J_out,
                    double* dJ_dcs, double* dJ_dsct, double* dJ_dchi0_dev);

/* Measurement utility (not part of the method): copies `bytes` (a multiple of
 * 16) from src_dev to dst_dev with a plain streaming kernel on hip_stream --
 * the achievable read+write HBM ceiling against which the step kernel's
 * bandwidth is compared. Asynchronous. LBM_EINVAL on NULL pointers or a size
 * that is not a multiple of 16. */
int lbm_stream_copy(void* dst_dev, const void* src_dev, size_t bytes, void* hip_stream);

const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
