/*
 * lbm.h - C ABI of the MI355X (gfx950) MRT lattice Boltzmann library with the Yu and
 * Chai strain-rate formulas.
 *
 * Method: Zhang, Huang, Wang, Shi, "The computation of strain rate tensor in
 * multiple-relaxation-time lattice Boltzmann model" (arXiv 1704.07559).
 *   - the He-Luo D3Q19 MRT model of Section 2 (Eqs. mrteq, edf, omega, HeLuoD3Q19, the
 *     matrix T, Eqs. meq, sD3Q15, sD3Q15meaning);
 *   - the Yu formula (Eq. LuoS) and the Chai formula (Eq. ChaiS) of Section 3;
 *   - the D2Q9 and D3Q15 variants that Section 5.3 says the Chai formula covers, with the
 *     Yu-type formulas obtained by the route of Section 5.4 (the D2Q9 basis is the
 *     Lallemand-Luo one, the D3Q15 basis the d'Humieres et al. 2002 one; the paper gives
 *     neither).
 *
 * Conventions shared by every entry point
 *   - All arrays are structure-of-arrays, x fastest: element (c, z, y, x) of a field with
 *     C components sits at  c*N + (z*ny + y)*nx + x,  N = nx*ny*nz.
 *   - Populations are the deviations g_i = f_i - w_i rho0 (the delta-rho form of Eq. edf),
 *     i in the velocity order of Eq. HeLuoD3Q19 (D3Q19), (0, E, N, W, S, NE, NW, SW, SE)
 *     (D2Q9), or (0, +x, -x, +y, -y, +z, -z, (+++), (---), (++-), (--+), (+-+), (-+-),
 *     (-++), (+--)) (D3Q15). "Canonical" populations are the pre-collision g_i(x, n) of
 *     Eq. mrteq, as a Q-component field. The two state buffers use the library's own
 *     layout (row-interleaved post-collision populations, element (i, z, y, x) at
 *     ((z*ny + y)*Q + i)*nx + x); only lbm_get_populations / lbm_set_populations /
 *     lbm_init convert, and lbm_save_state / lbm_load_state copy it as it is.
 *   - Strain fields hold 6 components (xx, yy, zz, xy, yz, xz) for D3Q19 and D3Q15 and 3
 *     components (xx, yy, xy) for D2Q9, of the strain of the pre-collision state.
 *   - Lattice units: delta_x = delta_t = 1, c_s^2 = 1/3.
 *   - Every pointer argument named as a field is a DEVICE pointer, caller-owned, and must
 *     stay valid while the context uses it. Population buffers must be 256-byte aligned,
 *     other fields 4-byte aligned. No entry point allocates device memory except lbm_init
 *     (a small reduction scratch) and none frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Every call is
 *     asynchronous on that stream, except where a host result is returned (lbm_reduce,
 *     lbm_strain_loss_seed), which synchronise the stream before returning
 *     (lbm_reduce_async is the non-blocking form of lbm_reduce).
 *   - No C++ exception crosses the ABI. Every call returns an lbm_status; on failure
 *     lbm_last_error() gives a message (thread-local). Arguments are validated before any
 *     launch; a kernel-launch failure maps to LBM_EHIP.
 *   - A context is not thread-safe; use one per stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,       /* invalid argument (sizes, alignment, aliasing, enum values) */
  LBM_EHIP = -2,         /* a HIP runtime call or kernel launch failed */
  LBM_ENOMEM = -3,       /* device scratch allocation failed */
  LBM_ESTATE = -4,       /* call not valid in the context's state (e.g. no force field) */
  LBM_ENONFINITE = -5,   /* lbm_reduce found non-finite populations */
  LBM_EUNSUPPORTED = -6  /* valid but not provided combination (e.g. the D2Q9 adjoint) */
} lbm_status;

typedef enum { LBM_D2Q9 = 9, LBM_D3Q15 = 15, LBM_D3Q19 = 19 } lbm_lattice;
typedef enum { LBM_F32 = 0, LBM_F16 = 1, LBM_BF16 = 2 } lbm_storage;
typedef enum { LBM_STRAIN_NONE = 0, LBM_STRAIN_YU = 1, LBM_STRAIN_CHAI = 2 } lbm_strain_kind;
typedef enum {
  LBM_VISC_CONST = 0,
  LBM_VISC_SMAGORINSKY = 1,
  LBM_VISC_POWERLAW = 2,
  LBM_VISC_SMAGORINSKY_IMPLICIT = 3
} lbm_visc_kind;

/*
 * Model parameters.
 *  s[]        diagonal of Lambda-hat (Eq. sD3Q15): 19 entries for D3Q19, the first 9 for
 *             D2Q9 (rates of rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy), the first 15 for
 *             D3Q15 (rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, p_ww, p_xy, p_yz,
 *             p_xz, m_xyz). The s_nu slots (D3Q19: 9, 11, 13, 14, 15; D3Q15: 9..13;
 *             D2Q9: 7, 8) must hold one value, the initial s_nu.
 *  omega_*    the free equilibrium coefficients of Eq. meq (paper: 3, -11/2, -1/2);
 *             D3Q19 only.
 *  visc_kind  LBM_VISC_CONST: s_nu fixed.  LBM_VISC_SMAGORINSKY: nu = nu0 + c_smag^2 |S|.
 *             LBM_VISC_POWERLAW: nu = clamp(K_pl |S|^(n_pl-1), nu_min, nu_max), with
 *             nu = nu_max (n_pl < 1) or nu_min (n_pl > 1) at |S| = 0. |S| = sqrt(2 S:S).
 *             s_nu = 1/(3 nu + 1/2) relaxes the collision; the strain of the next step
 *             uses the s_nu of the previous collision at the node (held in s_nu_field).
 *             LBM_VISC_SMAGORINSKY_IMPLICIT (every lattice): no lagged field; every node
 *             solves s_nu = 1/(3 (nu0 + c_smag^2 |S(s_nu)|) + 1/2), S(s_nu) being the strain
 *             formula (affine in s_nu) at the rate of this very collision; s_nu_field may be
 *             NULL.
 *  visc_strain which formula drives the viscosity (LBM_STRAIN_YU or LBM_STRAIN_CHAI).
 *  walls_y    0: periodic in y. 1: halfway bounce-back walls at y = -1/2 and y = ny - 1/2.
 *  force[3]   uniform body force (Guo forcing, j = sum c g + F/2) used when
 *             force_field is NULL; force_field: device float[3*N] field, or NULL.
 *  strain_force_correction  1: every strain the library computes (emitted by lbm_step,
 *             lbm_strain, lbm_reduce, the strain driving the viscosity) takes the force-
 *             corrected non-equilibrium part, m - m^eq + S_F/2 (Yu) or f - f^eq + F-bar/2
 *             (Chai), S_F = T F-bar the Guo source in moment space. This is the force effect
 *             Section 1 attributes to Premnath et al., obtained from the first-order
 *             Chapman-Enskog balance of the forced collision; it removes the u F terms the
 *             force puts into the second-order moments. No effect without a force. The adjoint
 *             entry points differentiate it. 0: the plain non-equilibrium part.
 */
typedef struct {
  int lattice;       /* lbm_lattice */
  int storage;       /* lbm_storage of the population buffers */
  int nx, ny, nz;    /* nz = 1 for D2Q9 */
  int walls_y;
  double rho0;
  double s[19];
  double omega_eps, omega_epsj, omega_xx;
  int visc_kind;     /* lbm_visc_kind */
  int visc_strain;   /* lbm_strain_kind */
  double nu0, c_smag, K_pl, n_pl, nu_min, nu_max;
  double force[3];
  const float* force_field;
  int strain_force_correction; /* 0 or 1, see above */
} lbm_params;

/* sizeof(lbm_params) as the library was built: a binding that mirrors the struct (ctypes,
 * another language) checks its own layout against it before the first call. */
size_t lbm_params_size(void);

/* Bytes of one population buffer (Q * N * element size) for these parameters, or 0 if the
 * parameters are invalid. */
size_t lbm_population_bytes(const lbm_params* p);

/*
 * Create a context over caller-owned device buffers and write the initial state.
 *  f_a, f_b     two distinct population buffers of lbm_population_bytes(p) bytes.
 *  s_nu_field   device float[N]; required for LBM_VISC_SMAGORINSKY and LBM_VISC_POWERLAW
 *               (may be NULL otherwise). Filled with the initial s_nu. For D2Q9 boxes that
 *               take two steps per launch (see lbm_step) the context allocates a second
 *               float[N] for the field between the two launches of a four-step group.
 *  rho_u        device float[4*N]: planes delta_rho, u_x, u_y, u_z (u_z ignored for D2Q9);
 *               NULL = fluid at rest. Initial populations are g^eq(delta_rho, rho0 u)
 *               (the delta-rho form of Eq. edf).
 *  grad_u       device float[9*N], plane a*3+b = d u_b / d x_a, or NULL. When given, the
 *               non-equilibrium moments predicted by Eq. YuLuobasis are added (D3Q19: rows
 *               1, 9, 11, 13, 14, 15; D2Q9: rows 1, 7, 8; D3Q15: rows 1, 9..13, the
 *               inverse of its Yu-type formula), so the strain of the initial state equals
 *               the symmetric part of grad_u.
 * Errors: LBM_EINVAL (bad sizes, alignment, aliasing, unequal s_nu slots), LBM_ENOMEM,
 * LBM_EHIP. On error *out is NULL.
 */
lbm_status lbm_init(lbm_ctx** out, const lbm_params* p, void* f_a, void* f_b, float* s_nu_field,
                    const float* rho_u, const float* grad_u, void* stream);

/*
 * Advance nsteps steps of Eq. mrteq (collide with moment-space relaxation, Eq. mrteqvT,
 * then pull streaming), one fused kernel per step. D2Q9 on boxes at least 256 nodes wide
 * (periodic, or with walls in y) takes its steps in groups of four as two launches of two steps each (the intermediate level never leaves the
 * chip; half the HBM traffic); the remaining steps run singly. The result is the same, bit for
 * bit, as that of nsteps single steps.
 *  S_out        device float[6*N] (D3Q19, D3Q15) / [3*N] (D2Q9) or NULL: receives, at every step
 *               (at the second step of a launch of two), the strain (formula `strain_kind`) of
 *               that step's pre-collision state; after the call it holds the strain of the
 *               state at level n_end - 1.
 *  strain_kind  LBM_STRAIN_YU or LBM_STRAIN_CHAI (ignored when S_out is NULL).
 *  save         device float[nsteps*R*N] or NULL, R = lbm_save_planes(ctx) (D3Q19 only;
 *               LBM_EUNSUPPORTED otherwise):
 *               step k writes at offset k*R*N the record its adjoint needs: planes 0..2 the
 *               momentum j = sum c g + F/2 its collision used; for a strain-dependent
 *               viscosity (R = 10) also planes 3..8, the non-equilibrium moments
 *               m - m^eq of rows 1, 9, 11, 13, 14, 15 that enter Eq. LuoS (plus S_F/2 with
 *               strain_force_correction), and plane 9, the
 *               s_nu its strain was taken with (the lagged field value, or the implicitly
 *               solved rate).
 * Only kernel launches are queued on `stream` (no allocation, copy or wait), so calls can be
 * captured into a HIP graph. The context alternates its two population buffers on the host
 * at every launch, and a call of an even number of steps leaves the state in the buffer it
 * started from: a captured sequence must hold an even number of steps for each replay to
 * start from the buffer the capture started from, and lbm_step_count counts the captured
 * steps only.
 */
lbm_status lbm_step(lbm_ctx* ctx, int nsteps, float* S_out, int strain_kind, float* save, void* stream);

/* Planes per step of lbm_step's adjoint record: 3 (constant viscosity) or 10 (strain-dependent
 * viscosity); 0 where the adjoint is not provided (D2Q9, D3Q15) or for a NULL context. */
int lbm_save_planes(const lbm_ctx* ctx);

/* Planes of the adjoint state lam (each N floats): 19 (the populations), or 20 for the lagged
 * viscosity kinds, whose plane 19 is the adjoint of the s_nu field; 0 where the adjoint is not
 * provided (as lbm_save_planes) or for NULL. */
int lbm_adjoint_planes(const lbm_ctx* ctx);

/* Strain of the current pre-collision state by the Yu (Eq. LuoS) or Chai (Eq. ChaiS)
 * formula, with the current s_nu field, into S_out (device float[6*N] / [3*N]). */
lbm_status lbm_strain(lbm_ctx* ctx, int strain_kind, float* S_out, void* stream);

/*
 * Global diagnostics of the current state, accumulated in FP64 with a deterministic
 * two-pass reduction. The collision conserves mass and momentum exactly (the conserved rows
 * of Eq. solvem, Eq. continuityandmomentum: delta-rho and j are unchanged by the relaxation,
 * and the Guo force adds F per node and step), so [0] and [1..3] watch the run's round-off;
 * [5] is the dissipation measure the strain formulas (Eq. LuoS, Eq. ChaiS) feed.
 * host_out (host memory, 8 doubles):
 *   [0] sum delta_rho  [1..3] sum j (j includes F/2)  [4] sum |j|^2/(2 rho0)
 *   [5] sum S:S (Yu, off-diagonals counted twice)  [6] max |j|/rho0  [7] count of
 *   non-finite populations.
 * Synchronises the stream. Returns LBM_ENONFINITE (after filling host_out) if [7] > 0.
 */
lbm_status lbm_reduce(lbm_ctx* ctx, double* host_out, void* stream);

/*
 * The same diagnostics without waiting: the two reduction passes and a copy of the 8
 * doubles into `out` are queued on `stream` and the call returns at once. `out` is device
 * memory or pinned (page-locked) host memory, 8-byte aligned; its values are valid once the
 * stream has passed this point (an event or a later synchronisation). The non-finite count
 * is not checked here: the caller reads out[7]. The reduction scratch belongs to the
 * context, so reductions of one context must be ordered (one stream, or synchronised
 * between streams). Lets a run keep the GPU busy while it monitors the state every k steps.
 * Errors: LBM_EINVAL (NULL or misaligned out), LBM_EHIP.
 */
lbm_status lbm_reduce_async(lbm_ctx* ctx, double* out, void* stream);

/* Current canonical pre-collision populations g_i(x, n) as FP32 (device float[Q*N]). */
lbm_status lbm_get_populations(lbm_ctx* ctx, float* f_canon, void* stream);

/* Replace the state by canonical populations (device float[Q*N]), rounded to the storage
 * type. The s_nu field is left as it is. */
lbm_status lbm_set_populations(lbm_ctx* ctx, const float* f_canon, void* stream);

/* Checkpoint support: lbm_state_bytes() bytes hold the internal population buffer and,
 * for a variable viscosity, the s_nu field. save/load are device-to-device copies. */
size_t lbm_state_bytes(const lbm_ctx* ctx);
lbm_status lbm_save_state(lbm_ctx* ctx, void* dst, void* stream);
lbm_status lbm_load_state(lbm_ctx* ctx, const void* src, void* stream);
long long lbm_step_count(const lbm_ctx* ctx);
lbm_status lbm_set_step_count(lbm_ctx* ctx, long long n);

/*
 * Discrete adjoint (D3Q19, periodic or walls_y, any viscosity kind; the paper has no adjoint).
 * For one forward step g^{n+1} = P C(g^n, F) (C the collision, P the pull streaming), given
 * lam_in = dJ/d(state^{n+1}) and rec_n, the record lbm_step's `save` wrote for step n
 * (device float[lbm_save_planes(ctx)*N]), writes
 *   lam_out = (dC/dg)^T P^T lam_in              (device float[A*N], A = lbm_adjoint_planes)
 * and, if grad_force is not NULL, accumulates (dC/dF)^T P^T lam_in into it (device
 * float[3*N], read-modify-write). lam planes 0..18 are populations in canonical layout.
 * Strain-dependent viscosity: the collision rate s_new is a function of the strain of
 * Eq. LuoS (lagged: of the state and the s_nu field; implicit: solved with the strain), and
 * its derivative enters the transpose; for the lagged kinds plane 19 of lam_in is dJ/d(s_nu
 * field of step n+1) and plane 19 of lam_out dJ/d(s_nu field of step n). The power-law clamps
 * and |S| = 0 take a zero derivative. lam_in and lam_out must not alias.
 */
lbm_status lbm_adjoint_step(lbm_ctx* ctx, const float* rec_n, const float* lam_in, float* lam_out,
                            float* grad_force, void* stream);

/*
 * nsteps reverse steps in one call: for n = nsteps-1 down to 0, lbm_adjoint_step with the
 * record rec + n*R*N (R = lbm_save_planes(ctx), as one lbm_step(nsteps, ..., save) call
 * wrote them), the adjoint state ping-ponging between lam_a and lam_b (each device
 * float[lbm_adjoint_planes(ctx)*N], not overlapping). On entry lam_a holds the adjoint after
 * the last step; on return lam_a holds the adjoint before the first (lam_b is scratch: the
 * states between the first and the last step are kept with planes 0..18 in the
 * row-interleaved order of the population buffers, and its contents on return are
 * unspecified). The result equals nsteps lbm_adjoint_step calls bit for bit.
 * grad_force as in lbm_adjoint_step. Saves a host round trip per step.
 */
lbm_status lbm_adjoint_steps(lbm_ctx* ctx, int nsteps, const float* rec, float* lam_a, float* lam_b,
                             float* grad_force, void* stream);

/*
 * lbm_adjoint_steps without the lam_b workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc). The
 * reverse sweep ping-pongs between `lam` (device float[lbm_adjoint_planes(ctx)*N]: on entry
 * the adjoint after the last step, on return the adjoint before the first) and a fixed
 * scratch of 64 MiB that the library holds on every device it runs on (a static device
 * array, not allocated by this call), so A*N*4 bytes must not exceed 64 MiB (A =
 * lbm_adjoint_planes: about 838 000 nodes with 20 planes). rec and grad_force as in
 * lbm_adjoint_steps; the result equals lbm_adjoint_steps' bit for bit. The call allocates
 * nothing: it validates, takes the scratch address of the stream's device (looked up once
 * per device, by lbm_init on its stream's device or else by the first call here), and queues
 * the kernel launches and, for an odd nsteps, one device-to-device copy into lam, so it can be
 * captured into a HIP graph. Every call on one device shares that device's scratch, which keeps the last
 * call's contents (every step overwrites it whole, so nothing needs clearing): calls that
 * overlap on one device (several streams, several host threads) race and must be ordered by
 * the caller. Errors: LBM_EINVAL (NULL or misaligned pointers, nsteps < 0, the state larger
 * than the scratch), LBM_EUNSUPPORTED (D2Q9, D3Q15), LBM_EHIP.
 */
lbm_status lbm_adjoint_steps_noalloc(lbm_ctx* ctx, int nsteps, const float* rec, float* lam, float* grad_force,
                                     void* stream);

/*
 * Loss J = sum_x S:S of the current pre-collision state (Yu formula, which equals Chai,
 * Section 5.1, at the rate the viscosity model gives the state: s_nu of the parameters, the
 * lagged field, or the implicitly solved rate), its gradient into lam_out (device
 * float[lbm_adjoint_planes(ctx)*N]: dJ/dg in canonical layout, plus dJ/d(s_nu field) in
 * plane 19 for the lagged kinds), and, if grad_force is not NULL, dJ/dF (through
 * j = sum c g + F/2) added into grad_force. J is accumulated in FP64 and written to *J_host.
 * Synchronises the stream.
 */
lbm_status lbm_strain_loss_seed(lbm_ctx* ctx, float* lam_out, float* grad_force, double* J_host, void* stream);

/*
 * Adjoint of the initial state g^0 = g^eq(0, rho0 u0): grad_u0 (device float[3*N]) =
 * sum_i lam0_i dg^eq_i/du at u0 (rho_u: device float[4*N] as given to lbm_init). Only planes
 * 0..18 of lam0 are read (the initial s_nu field does not depend on u0).
 */
lbm_status lbm_init_adjoint(lbm_ctx* ctx, const float* rho_u, const float* lam0, float* grad_u0, void* stream);

/*
 * STREAM-style copy of `bytes` bytes from src to dst (device pointers, 16-byte aligned,
 * bytes a multiple of 16, the ranges not overlapping), 16-byte nontemporal loads and stores,
 * asynchronous on `stream`. A measurement aid, not part of the method: it gives the
 * achievable HBM bandwidth of a pure streaming pattern on the device, the practical ceiling
 * of the step kernel (whose algorithmic traffic is the same read-once/write-once streams).
 * Errors: LBM_EINVAL (NULL, misaligned, overlapping, bytes not a multiple of 16), LBM_EHIP.
 */
lbm_status lbm_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

void lbm_destroy(lbm_ctx* ctx);
const char* lbm_status_string(int status);
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
