/*
 * pm.h -- C-ABI of the MI355X particle-mesh hot path (libpm.so).
 *
 * Li et al., "Differentiable Cosmological Simulation with the Adjoint Method"
 * (arXiv:2211.09815): the particle-mesh force (Sec. 2.2), its vector-Jacobian
 * product (Sec. 3.6), the FastPM kick-drift-kick leapfrog (Sec. 2.3,
 * eq. KDFK) and its adjoint with reverse-time integration (Sec. 3.6,
 * eqs. KDFKO_adj and KDFKO_grad), the 2LPT initial conditions (Sec. 2.1,
 * eq. lpt), the final-density objective of Sec. 4.2, and the light-cone
 * observation of Sec. 2.4 with the adjoint of an objective on the
 * observables (Sec. 3.4).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Return value: PM_OK (0) or a negative PM_E* code.  Arguments are checked
 *    before anything is launched; no call aborts, throws or exits.  The text
 *    of the last error of a plan is returned by pm_last_error(plan)
 *    (pm_last_error(NULL) gives the last plan-creation error of the calling
 *    thread).
 *  - Units: positions, displacements and momenta are in mesh cells, time in
 *    1/H0 (H0 = 1).  Calls that evaluate the force take `omega_m` (> 0) and
 *    form the Poisson coefficient 1.5 * Omega_m themselves (the Poisson
 *    equation for phi~ = a phi, Sec. 2.2); their derivative outputs are with
 *    respect to Omega_m.
 *  - Particles: N_p = ptcl[0]*ptcl[1]*ptcl[2] in row-major lattice order.
 *    Particle n = (i*ptcl[1] + j)*ptcl[2] + k sits at the Lagrangian position
 *    q = (i, j, k) * r + lattice_offset with r[a] = mesh[a] / ptcl[a]; only
 *    its displacement s is stored (x = q + s, Sec. 2.1).  Per-particle
 *    vectors are structure-of-arrays [3][N_p] (all x components first).
 *  - Mesh: real fields [mesh[0]][mesh[1]][mesh[2]] in C order (last index
 *    contiguous); half spectra [mesh[0]][mesh[1]][mesh[2]/2 + 1] of
 *    interleaved complex numbers (re, im), exactly numpy's rfftn layout.
 *  - Types: "state" arrays (displacement s, momentum p) have
 *    cfg.state_dtype; mesh fields, spectra, accelerations, weights and the
 *    adjoint variables (xi, pi, alpha) have cfg.mesh_dtype.
 *  - Ownership: the caller owns every pointer argument; all pointers except
 *    host-struct arguments are DEVICE pointers on the plan's device.  The
 *    plan owns only its scratch (meshes, spectra, twiddles, reduction space,
 *    one [3][N_p] mesh-dtype array for the native adjoint loop),
 *    allocated once in pm_plan_create, plus the 2LPT lattice scratch:
 *    with cfg.lpt_scratch = 1 pm_plan_create allocates it too, and then no
 *    call allocates; with 0 the first pm_lpt / pm_lpt_vjp call does.
 *    pm_workspace_bytes reports both.  The other calls allocate nothing.
 *  - Streams: every call is asynchronous on the given stream (0 = default).
 *    Scalars reported on the device (J, omega_m_bar, theta_bar) are ready after
 *    the stream is synchronised.  A plan is not thread-safe; calls made with
 *    one plan on different streams must be ordered by the caller.
 *  - Determinism: with cfg.deterministic = 1 the paint sums each mesh tile
 *    in 64-bit fixed point with a per-tile binary scale, so painted meshes,
 *    forces and every particle output are bitwise reproducible (GPU float
 *    atomics are not; the paper's Table rep discusses that effect).  Only
 *    the FP64 per-tile partial sums behind theta_bar depend on the order of
 *    particles within a tile, at the 1e-15 relative level.  With
 *    cfg.deterministic = 0 the paint uses floating-point LDS atomics.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PM_OK            0
#define PM_EINVAL       -1   /* bad argument value or NULL pointer           */
#define PM_ESHAPE       -2   /* mesh or lattice shape not supported          */
#define PM_ENOMEM       -3   /* device allocation failed (plan creation)     */
#define PM_EDEVICE      -4   /* a HIP call failed                            */
#define PM_EUNSUPPORTED -5   /* valid but not implemented combination        */
#define PM_ENONFINITE   -6   /* NaN/Inf found by pm_check_finite             */

#define PM_F32 0
#define PM_F64 1

/* ---- plan -------------------------------------------------------------- */
typedef struct pm_plan_s* pm_plan;

typedef struct {
    int32_t mesh[3];        /* mesh cells per axis: powers of two, 4..1024     */
    int32_t ptcl[3];        /* particle lattice per axis (>= 1); for pm_lpt    */
                            /* and pm_lpt_vjp a cube with a power-of-two side  */
    double  box[3];         /* box side in Mpc/h (only pm_lpt/pm_lpt_vjp use it) */
    double  lattice_offset; /* offset of the lattice in mesh cells (all axes)  */
    int32_t mesh_dtype;     /* PM_F32 or PM_F64: mesh, FFT, force, adjoint     */
    int32_t state_dtype;    /* PM_F32 or PM_F64: s and p accumulators          */
    int32_t deterministic;  /* 1: the paint sums each tile in 64-bit fixed     */
                            /* point (integer LDS atomics, associative), so    */
                            /* every mesh and particle output is bitwise       */
                            /* reproducible; 0: it sums in the mesh type with  */
                            /* floating-point LDS atomics, whose order and so  */
                            /* rounding change from run to run (Table rep of   */
                            /* the paper discusses that effect)                */
    int32_t lpt_scratch;    /* 1: pm_plan_create also allocates the 2LPT       */
                            /* lattice scratch (ptcl must then be a power-of-  */
                            /* two cube in 4..1024 and box a positive cube),   */
                            /* so pm_lpt and pm_lpt_vjp allocate nothing; 0:   */
                            /* the first of those calls allocates it           */
    int32_t lpt_keep;       /* 1: pm_lpt keeps the second-order fields it      */
                            /* forms (the Hessian of the first-order potential */
                            /* and the second-order displacement) in the 2LPT  */
                            /* scratch, and the next pm_lpt_vjp uses them when */
                            /* it gets the same omega pointer and bytewise the */
                            /* same cosmology and coefficients, instead of     */
                            /* forming them again; the caller must not change  */
                            /* omega's contents in between.  Any pm_lpt_vjp    */
                            /* consumes them.  0: pm_lpt_vjp always forms them */
} pm_config;

/* Creates a plan on the current HIP device and allocates its scratch.
 * Errors: PM_EINVAL (NULL, a flag other than 0 or 1), PM_ESHAPE (mesh not a
 * power of two in 4..1024, a ptcl side outside 1..65536, more than 2^31
 * particles, lpt_scratch with a lattice 2LPT cannot use), PM_EUNSUPPORTED
 * (mesh_dtype F32 with state_dtype F64 is allowed; mesh F64 with state F32
 * is not), PM_ENOMEM, PM_EDEVICE. */
int pm_plan_create(const pm_config* cfg, pm_plan* out);
int pm_plan_destroy(pm_plan plan);
/* Bytes of device scratch a plan for cfg holds (0 if invalid): what
 * pm_plan_create allocates, plus, for a cubic lattice, the 2LPT lattice
 * scratch (allocated by pm_plan_create with cfg.lpt_scratch = 1, else by
 * the first pm_lpt / pm_lpt_vjp call). */
size_t pm_workspace_bytes(const pm_config* cfg);
const char* pm_last_error(pm_plan plan);
const char* pm_strerror(int code);

/* ---- a3: CIC paint (Sec. 2.2, eq. cic) --------------------------------- */
/* mesh[c][cell] = sum_n w_c(n) W(cell, q_n + disp_n) for c < nch, with the
 * trilinear weight W of eq. cic (base node floor(x), periodic wrap).
 * disp: [3][N_p] state dtype.  weights: [nch][N_p] mesh dtype, or NULL for
 * unit mass (then nch must be 1).  mesh: [nch][N_c] mesh dtype, overwritten.
 * 1 <= nch <= 4. */
int pm_paint(pm_plan plan, const void* disp, const void* weights, int nch,
             void* mesh, hipStream_t stream);

/* ---- a4/a6: 3-D real FFT on the mesh (Sec. 2.2) ------------------------ */
/* dir = +1: R2C, out(k) = sum_x in(x) exp(-i k.x) (unnormalised), in: batch
 * real fields, out: batch half spectra.  dir = -1: C2R, out(x) = (1/N_c)
 * sum_k in(k) exp(+i k.x) over the Hermitian completion of the half
 * spectrum (the imaginary parts on the kz = 0 and kz = N/2 planes are
 * ignored, as numpy's irfftn does); `in` is used as scratch and destroyed.
 * in and out must not overlap.  1 <= batch <= 4. */
int pm_fft(pm_plan plan, int dir, void* in, void* out, int batch, hipStream_t stream);

/* ---- a5: Poisson gradient (Sec. 2.2) ----------------------------------- */
/* grad_k[j](k) = T_j(k) delta_k(k), T_j = i k_j 1.5 omega_m / k^2, k_j =
 * 2 pi m_j / mesh[j]; zero at k = 0 and on the Nyquist plane of axis j (so
 * that each operator is real and exactly anti-self-adjoint).  delta_k: one
 * half spectrum; grad_k: [3] half spectra (must not overlap delta_k). */
int pm_poisson_grad(pm_plan plan, const void* delta_k, void* grad_k, double omega_m,
                    hipStream_t stream);

/* ---- a7: CIC readout (Sec. 2.2) ---------------------------------------- */
/* out[c][n] = sum_cell W(cell, q_n + disp_n) mesh[c][cell], the same weights
 * as pm_paint.  mesh: [nch][N_c], out: [nch][N_p], 1 <= nch <= 4. */
int pm_readout(pm_plan plan, const void* disp, const void* mesh, int nch, void* out,
               hipStream_t stream);

/* ---- a3..a7 composed: PM force ----------------------------------------- */
/* acc = -grad phi~ at the particles: paint, delta = rho N_c/N_p - 1, R2C,
 * Poisson gradient, 3 C2R, readout.  acc: [3][N_p] mesh dtype. */
int pm_force(pm_plan plan, const void* disp, double omega_m, void* acc, hipStream_t stream);

/* ---- a8: force VJP (Sec. 3.6; scatter/gather VJPs) ---------------------- */
/* For cotangent acc_bar [3][N_p] of the accelerations:
 *   disp_bar[k][n] = sum_j acc_bar[j][n] d a_j(n) / d x_k(n') summed over n'
 *                    (the VJP with respect to all particle positions),
 *   *omega_m_bar  += sum_{n,j} acc_bar[j][n] a_j(n) / omega_m   (device
 *                    double; a is proportional to Omega_m),
 *   acc_out        = a (optional, may be NULL).
 * disp_bar: [3][N_p] mesh dtype, overwritten. */
int pm_force_vjp(pm_plan plan, const void* disp, const void* acc_bar, double omega_m,
                 void* disp_bar, double* omega_m_bar, void* acc_out, hipStream_t stream);

/* ---- a1: step coefficients and KDK steps (Sec. 2.3, eq. KDFK) ------------ */
/* Step i (1-based) goes from a_{i-1} to a_i through a_{i-1/2}:
 *   Ka = K(t_{i-1}, t_{i-1}, t_{i-1/2}),  D = D(t_{i-1/2}, t_{i-1}, t_i),
 *   Kb = K(t_i, t_{i-1/2}, t_i), and their derivatives with respect to
 *   Omega_m (dKa, dD, dKb). */
typedef struct { double Ka, D, Kb, dKa, dD, dKb; } pm_step_coef;

typedef struct {
    void* s;     /* [3][N_p] state dtype, displacement (in/out)              */
    void* p;     /* [3][N_p] state dtype, momentum (in/out)                  */
    void* acc;   /* [3][N_p] mesh dtype, force cache a_n (optional)          */
} pm_state;

typedef struct {
    void* xi;    /* [3][N_p] mesh dtype, adjoint of x (in/out)               */
    void* pi;    /* [3][N_p] mesh dtype, adjoint of p (in/out)               */
} pm_adj;

/* Forward start: a_0 = F(x_0); p <- p_0 + a_0 first->Ka.
 * In: (s_0, p_0).  Out: (s_0, p_{1/2}). */
int pm_fwd_init(pm_plan plan, pm_state* st, const pm_step_coef* first, double omega_m,
                hipStream_t stream);

/* Forward step i with merged kicks:
 *   s_i = s_{i-1} + p_{i-1/2} D_i;  a_i = F(x_i);
 *   p  <- p_{i-1/2} + a_i (Kb_i + next->Ka)     (next = step i+1)
 * or, with next == NULL (last step), p_n = p_{n-1/2} + a_n Kb_n and a_n is
 * stored in st->acc when st->acc != NULL.
 * In: (s_{i-1}, p_{i-1/2}).  Out: (s_i, p_{i+1/2}) or (s_n, p_n). */
int pm_step_fwd(pm_plan plan, pm_state* st, const pm_step_coef* cur,
                const pm_step_coef* next, double omega_m, hipStream_t stream);

/* ---- a9/a10: adjoint with reverse-time integration (eq. KDFKO_adj) ------ */
/* theta_bar: device double[2], accumulated (+=): [0] dJ/dOmega_m, [1]
 * dJ/dsigma8 (the steps only touch [0]).  The Omega_m derivative covers both
 * the step coefficients (their d/dOmega_m in pm_step_coef) and the force,
 * which is proportional to Omega_m: zeta = (pi . a) / omega_m. */

/* Reverse start at t_n.  In: (s_n, p_n, acc = a_n or NULL to recompute),
 * (xi_n, pi_n).  Computes alpha_n, zeta_n = pi_n . da/d(x, Omega_m) at x_n,
 * then the kick back:  p <- p_n - a_n Kb_n,  xi <- xi_n + alpha_n Kb_n,
 * theta_bar[0] += (pi_n . a_n) dKb_n + zeta_n Kb_n.
 * Out: (s_n, p_{n-1/2}), (xi_{n-1/2}, pi_n). */
int pm_adj_init(pm_plan plan, pm_state* st, pm_adj* adj, const pm_step_coef* last,
                double omega_m, double* theta_bar, hipStream_t stream);

/* Reverse step i (i = n..1) with merged kicks:
 *   theta_bar[0] += (xi_{i-1/2} . p_{i-1/2}) dD_i
 *   s_{i-1} = s_i - p_{i-1/2} D_i;   pi_{i-1} = pi_i + xi_{i-1/2} D_i
 *   a, alpha, zeta at x_{i-1} (force and its VJP with cotangent pi_{i-1})
 *   K = Ka_i + prev->Kb (prev = step i-1), or Ka_i when prev == NULL
 *   p <- p - a K;   xi <- xi + alpha K
 *   theta_bar[0] += (pi_{i-1} . a)(dKa_i + prev->dKb) + zeta K
 * In: (s_i, p_{i-1/2}), (xi_{i-1/2}, pi_i).
 * Out: (s_{i-1}, p_{i-3/2}), (xi_{i-3/2}, pi_{i-1}), or at i = 1
 * (s_0, p_0), (xi_0, pi_0). */
int pm_step_adj(pm_plan plan, pm_state* st, pm_adj* adj, const pm_step_coef* cur,
                const pm_step_coef* prev, double omega_m, double* theta_bar,
                hipStream_t stream);

/* Whole loops (native drivers of the two calls above).  coefs: host array of
 * n steps.  pm_run_fwd = pm_fwd_init + n x pm_step_fwd;  pm_run_adj =
 * pm_adj_init + n x pm_step_adj (reverse order), with bitwise the same
 * result.  With st->acc given, the loops use it as scratch: each gather
 * stores a there and leaves its kick to the next step's drift (the plan's
 * workspace holds alpha for the adjoint).  After pm_run_fwd, acc holds a_n
 * as after the step calls; after pm_run_adj its contents are unspecified.
 * With st->acc given, pm_run_adj also holds adj->pi particle-major while it
 * runs (whenever 3 N_p values fit the plan's four meshes) and returns it as
 * [3][N_p]; if the call fails, pi's contents are unspecified. */
int pm_run_fwd(pm_plan plan, pm_state* st, const pm_step_coef* coefs, int n, double omega_m,
               hipStream_t stream);
int pm_run_adj(pm_plan plan, pm_state* st, pm_adj* adj, const pm_step_coef* coefs, int n,
               double omega_m, double* theta_bar, hipStream_t stream);

/* The reverse loop resumed from the point where pm_step_adj(n) would
 * continue, (s_n, p_{n-1/2}), (xi_{n-1/2}, pi_n), after pm_adj_init or any
 * pm_step_adj call: n reverse steps n..1 (coefs[0..n-1]), bitwise the same
 * as those n pm_step_adj calls.  For drivers that interleave their own work
 * with the last reverse steps (the light-cone gradient adds its bumps there)
 * and run the rest natively.  st->acc, if given, is scratch as in pm_run_adj,
 * and pi is handled as there.  Errors as pm_step_adj. */
int pm_run_adj_from(pm_plan plan, pm_state* st, pm_adj* adj, const pm_step_coef* coefs, int n,
                    double omega_m, double* theta_bar, hipStream_t stream);

/* ---- piecewise reverse from forward checkpoints (Sec. 3.5) ---------------- */
/* Where the reverse-time integration drifts too far from the forward
 * trajectory (long or strongly nonlinear runs, FP32 state), the backward
 * evolution can be resumed piecewise from states saved during the forward
 * pass.  Checkpoint j (1 <= j <= n) holds the state at which the reverse step
 * j starts: s_j and p_{j-1/2}.
 *   step[k]: host array, strictly increasing steps in [1, n];
 *   s[k], p[k]: host arrays of device buffers [3][N_p] in the state dtype,
 *   owned by the caller, written by pm_run_fwd_ckpt, read by pm_run_adj_ckpt.
 * count == 0 (or ck == NULL) makes both calls the plain loops. */
typedef struct {
    int count;
    const int* step;
    void* const* s;
    void* const* p;
} pm_checkpoints;

/* pm_run_fwd that also copies p_{j-1/2} (before step j) and s_j (after step
 * j) into checkpoint j.  Extra traffic: two state copies per checkpoint. */
int pm_run_fwd_ckpt(pm_plan plan, pm_state* st, const pm_step_coef* coefs, int n, double omega_m,
                    const pm_checkpoints* ck, hipStream_t stream);

/* pm_run_adj resuming from the checkpoints: the reverse step j + 1 lands its
 * drift on the stored s_j (the force and its VJP are evaluated there; the
 * theta term (xi . p) dD and pi += xi D are unchanged) and ends with p set to
 * the stored p_{j-1/2}; a checkpoint at n sets p_{n-1/2} after pm_adj_init.
 * xi and pi are integrated, and pi held, as in pm_run_adj.  With a checkpoint at every step
 * the adjoint runs on the forward trajectory itself.  Errors: PM_EINVAL for
 * unordered or out-of-range steps or NULL buffers (before any launch). */
int pm_run_adj_ckpt(pm_plan plan, pm_state* st, pm_adj* adj, const pm_step_coef* coefs, int n,
                    double omega_m, const pm_checkpoints* ck, double* theta_bar, hipStream_t stream);

/* ---- a11: objective and its VJP (Sec. 4.2) ------------------------------- */
/* delta = paint(x) N_c/N_p - 1; *J = (1/N_c) sum (delta - target)^2 (device
 * double, overwritten); disp_bar[k][n] = sum_cell dW/dx_k (2 (delta -
 * target)/N_p) (mesh dtype, overwritten; may be NULL). target: [N_c] mesh
 * dtype. */
int pm_density_mse(pm_plan plan, const void* disp, const void* target, double* J,
                   void* disp_bar, hipStream_t stream);

/* Density contrast of a unit-mass paint: delta = paint(x) N_c/N_p - 1
 * (the field the objective compares; [N_c] mesh dtype, overwritten). */
int pm_density(pm_plan plan, const void* disp, void* delta, hipStream_t stream);

/* ---- support: power spectrum (Sec. 2.1, eq. Plin) -------------------------- */
/* The paper defines P through <delta(k) delta(k')> = V P(k).  For the half
 * spectrum delta_k of a real field (pm_fft(+1); [n][n][n/2+1] mesh-dtype
 * complex, cubic mesh n^3 and cubic box L = cfg.box[0]), with the integer
 * wavevector m (k = 2 pi m / L), shell b = round(|m|) for b = 1..n/2:
 *   P[b-1]     = sum_shell w |delta_k V / N_c|^2 / V / sum_shell w,
 *   k[b-1]     = (2 pi / L) sum_shell w |m| / sum_shell w,
 *   count[b-1] = sum_shell w,
 * w = 2 for modes with 0 < mz < n/2 (each stands for its conjugate too) and
 * 1 on the mz = 0 and mz = n/2 planes.  No window deconvolution.  k, P,
 * count: device double [n/2], overwritten.  The shell sums are reduced in a
 * fixed order (no atomics), so repeated calls are bitwise equal.  Scratch:
 * the plan's spectrum buffers.  Errors: PM_EINVAL (NULL pointers),
 * PM_EUNSUPPORTED (mesh or box not cubic). */
int pm_power_spectrum(pm_plan plan, const void* delta_k, double* k, double* P, double* count,
                      hipStream_t stream);

/* Allocation-free form of pm_power_spectrum, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): no plan, and nothing is allocated or
 * freed.  Same estimator and outputs as pm_power_spectrum for a cubic mesh
 * of side n and box side `box` (Mpc/h); delta_k: [n][n][n/2+1] complex of
 * mesh_dtype (PM_F32 or PM_F64).  Its partial sums live in a static device
 * array of 12 MiB per GPU (held until the process ends), which covers every
 * mesh side up to 1024; a larger n is refused with PM_ESHAPE.  Every call on
 * one GPU uses that GPU's copy, so calls that overlap on one GPU (different
 * streams or threads) race; callers order them.  Errors (pm_last_error(NULL)):
 * PM_EINVAL, PM_ESHAPE, PM_EDEVICE. */
int pm_power_spectrum_noalloc(int n, double box, int mesh_dtype, const void* delta_k, double* k,
                              double* P, double* count, hipStream_t stream);

/* ---- support: cosmology tables (Appendix A, eqs. G_eval and Plin) --------- */
typedef struct {
    double omega_m, omega_b, h, n_s, sigma8, t_cmb;
} pm_cosmo;

/* Initial-condition factors at a_0: D1, D2 and P_m = a^2 E D_m' (momentum),
 * the amplitude A of P_lin(k) = A k^n_s T^2(k) (normalised to sigma8 at a=1),
 * each with its derivative with respect to Omega_m. */
typedef struct {
    double D1, D2, P1, P2, A;
    double dD1, dD2, dP1, dP2, dA;
} pm_ic_coef;

/* Host-only, FP64: growth ODEs in suppression-factor form (Appendix A),
 * G_D, G_K (eq. G_eval), the step coefficients of n steps on a_grid[0..n]
 * (midpoint half steps) with d/dOmega_m, and the IC factors at a_grid[0].
 * Either output may be NULL.  Flat LambdaCDM, H0 = 1. */
int pm_tables(const pm_cosmo* cosmo, const double* a_grid, int n, pm_step_coef* coefs,
              pm_ic_coef* ic);

/* ---- s1/s2: 2LPT initial conditions and VJP (Sec. 2.1, eq. lpt) ---------- */
/* omega: white noise on the ptcl^3 lattice ([N_p] mesh dtype, C order).
 * delta1 = irfft(sqrt(P(k)/V_cell) rfft(omega)), V_cell = (box/ptcl)^3;
 * s1 = -grad phi1, s2 = -grad phi2 with lattice spectral derivatives;
 * st->s = r (D1 s1 + D2 s2), st->p = r (P1 s1 + P2 s2) (state dtype). */
int pm_lpt(pm_plan plan, const void* omega, const pm_cosmo* cosmo, const pm_ic_coef* ic,
           pm_state* st, hipStream_t stream);

/* Transpose of pm_lpt: omega_bar = d<xi0, s_0> + <pi0, p_0> / d omega
 * ([N_p] mesh dtype, overwritten); theta_bar[0] += the Omega_m derivative
 * through P(k) and the time factors, theta_bar[1] += the sigma8 derivative.
 * xi0, pi0: adj->xi, adj->pi.  It forms the forward fields again, or, with
 * cfg.lpt_keep after a pm_lpt of the same omega pointer, cosmology and
 * coefficients, only the first-order ones (bitwise the same result). */
int pm_lpt_vjp(pm_plan plan, const void* omega, const pm_cosmo* cosmo,
               const pm_ic_coef* ic, const pm_adj* adj, void* omega_bar,
               double* theta_bar, hipStream_t stream);

/* ---- next 3: light-cone observation and its adjoint (Sec. 2.4, Sec. 3.4) -- */
/* Every particle is observed once, when it crosses the past light cone of an
 * observer at a = 1.  On step i (from a_{i-1} to a_i) its position is the
 * cubic Hermite spline in u = (a - a_{i-1}) / (a_i - a_{i-1}) through x and
 * dx/da = p w(a), w = 1 / (a^3 E(a)) (dx/dt = p / a^2, Sec. 2.3), at both
 * ends (x = q + s unwrapped, p the integer-time momenta); the light front
 * chi(a) = (c/H0) int_a^1 da' / (a'^2 E(a')) (comoving distance, in cells)
 * is the cubic Hermite spline through chi and dchi/da at both ends.  With
 * f(u) = |x(u) - observer| - chi(u), the particle is observed in step i when
 * f(0) < 0 <= f(1), at the root u* of f (safeguarded Newton); it records
 * x^ = x(u*), p^ = a^3 E(a^) dx/da(u*) and a^ = a_{i-1} + u* (a_i - a_{i-1}).
 * One copy of the periodic box is observed (no images). */

/* Light-front and velocity factors at one scale factor, with d/dOmega_m. */
typedef struct {
    double a;
    double chi;       /* cells */
    double dchi;      /* d chi / d a */
    double w;         /* 1 / (a^3 E(a)) */
    double chi_om, dchi_om, w_om;
} pm_lc_coef;

/* One observation step: the factors at a_{i-1} (c0) and a_i (c1). */
typedef struct {
    pm_lc_coef c0, c1;
    double omega_m;
    double observer[3];   /* cells, same frame as q + s */
    int32_t step;         /* i >= 1, written to obs_step of observed particles */
} pm_lc_step;

/* Host-only, FP64: out[k] for a_grid[0..n] (n + 1 entries), for a mesh cell
 * of `cell` Mpc/h (c/H0 = 2997.92458 Mpc/h).  chi by 8-point Gauss-Legendre
 * panels in sqrt(a'), Omega_m derivatives by dual numbers.  Returns
 * PM_EINVAL for NULL arguments, a outside (0, 1] or cell <= 0. */
int pm_lightcone_tables(const pm_cosmo* cosmo, const double* a_grid, int n, double cell,
                        pm_lc_coef* out);

/* Observation of step st->step.  s0, p0, s1, p1: [3][N_p] state dtype, the
 * displacements and integer-time momenta at a_{i-1} and a_i.  For every
 * particle observed in this step: obs[0..2][n] = x^, obs[3..5][n] = p^,
 * obs[6][n] = a^ ([7][N_p] state dtype) and obs_step[n] = st->step (int32
 * [N_p]); other particles' entries are left as they are.  *count (device
 * double) += the number observed.  Errors: PM_EINVAL for NULL buffers, a
 * step < 1 or c0.a >= c1.a. */
int pm_lightcone(pm_plan plan, const pm_lc_step* st, const void* s0, const void* p0,
                 const void* s1, const void* p1, void* obs, int32_t* obs_step,
                 double* count, hipStream_t stream);

/* *r_max (device double) = the largest comoving distance |q + disp -
 * observer| over the particles, in mesh cells, with the unwrapped positions
 * of the observation (disp: [3][N_p] state dtype; observer: host double[3]).
 * The light front only moves inward, at the speed of light, so a particle
 * outside it stays outside: once every particle is inside the front of
 * a_m (r_max < chi(a_m)), none has crossed in steps 1..m, and a driver may
 * run those steps without observing them.  NaN if a distance is.  Errors:
 * PM_EINVAL for NULL or non-finite arguments. */
int pm_lightcone_reach(pm_plan plan, const void* disp, const double* observer, double* r_max,
                       hipStream_t stream);

/* Transpose of pm_lightcone for the particles with obs_step[n] == st->step,
 * given the cotangent obs_bar ([7][N_p] mesh dtype) of (x^, p^, a^): adds
 * dJ/dx and dJ/dp at a_{i-1} to x0_bar, p0_bar and at a_i to x1_bar, p1_bar
 * ([3][N_p] mesh dtype each, +=; any may be NULL to skip it) and the
 * Omega_m derivative through chi, w and E to theta_bar[0] (device double,
 * +=).  The root is solved again on the given states, so they must be the
 * ones observed (or their reverse-time reconstruction).  The dependence of
 * u* on the states and on Omega_m is included (implicit function theorem). */
int pm_lightcone_vjp(pm_plan plan, const pm_lc_step* st, const void* s0, const void* p0,
                     const void* s1, const void* p1, const int32_t* obs_step,
                     const void* obs_bar, void* x0_bar, void* p0_bar, void* x1_bar,
                     void* p1_bar, double* theta_bar, hipStream_t stream);

/* The adjoint's bump at integer time k (Sec. 3.4; eq. explicit_adj adds
 * dJ/dz_k there).  p_k = p_{k-1/2} + a_k Kb_k, so a cotangent p_bar of p_k
 * also reaches a_k:
 *   xi += x_bar + Kb c,  pi += p_bar,
 *   theta_bar[0] += dKb sum(p_bar . acc) + Kb (*omega_m_bar),
 * where c and *omega_m_bar are pm_force_vjp's disp_bar and omega_m_bar for
 * the cotangent p_bar at x_k, and acc = a_k.  c, acc and omega_m_bar may be
 * NULL (Kb = 0: p_0, or a kick the caller's own VJP already covers).  p_bar
 * may be NULL (only xi += x_bar + Kb c; pi may then be NULL too, acc must
 * be).  xi, pi, x_bar, p_bar, c, acc: [3][N_p] mesh dtype. */
int pm_adj_bump(pm_plan plan, void* xi, void* pi, const void* x_bar, const void* p_bar,
                const void* c, double Kb, double dKb, const void* acc,
                const double* omega_m_bar, double* theta_bar, hipStream_t stream);

/* The truncated adjoint of Sec. 3.4, which sets a particle's adjoint to zero
 * after its crossing, in the discrete form this library gives it: the force
 * at integer time t_m takes the particles observed in steps 1..m as constant
 * sources, so its VJP gives them nothing (their own momentum cotangent
 * still acts).  A driver applies it to what a force VJP at t_m adds to the
 * position adjoint: x[c][n] = 0 for c < 3 and every particle with
 * 0 < obs_step[n] <= last (x: [3][N_p] mesh dtype, in place; obs_step as
 * pm_lightcone writes it; last < 1 does nothing).  The result is the exact
 * gradient of that modified forward map, not of the observed run. */
int pm_lightcone_truncate(pm_plan plan, void* x, const int32_t* obs_step, int32_t last,
                          hipStream_t stream);

/* The kick and drift operators of eq. KDFK on their own (out may alias the
 * input): p_out = p + acc K (p, p_out state dtype, acc mesh dtype) and
 * s_out = s + p D (state dtype).  The light-cone driver uses them for the
 * integer-time momenta and the reverse-time reconstruction one step ahead. */
int pm_kick(pm_plan plan, const void* p, const void* acc, double K, void* p_out,
            hipStream_t stream);
int pm_drift(pm_plan plan, const void* s, const void* p, double D, void* s_out,
             hipStream_t stream);

/* ---- support: health check and timing ------------------------------------ */
/* Sets *bad (device int) to 1 if any of n values of dtype in `x` is NaN or
 * Inf (else leaves it).  Returns PM_OK; the caller reads *bad after sync. */
int pm_check_finite(pm_plan plan, const void* x, int64_t n, int dtype, int* bad,
                    hipStream_t stream);

/* STREAM-like bandwidth kernels (measurement support): the HBM rate of a
 * pure read of nbytes at src (mode PM_STREAM_READ), of a copy src -> dst
 * (PM_STREAM_COPY) and of a pure write of zeros to dst (PM_STREAM_WRITE),
 * with 16-byte vectors in grid-stride loops over 2048 workgroups.  nbytes: a
 * positive multiple of 16; src and dst 16-byte aligned device pointers, not
 * overlapping.  The caller times the call (e.g. with events on `stream`).
 * Errors: PM_EINVAL for a bad mode, size or pointer. */
#define PM_STREAM_READ  0
#define PM_STREAM_COPY  1
#define PM_STREAM_WRITE 2
int pm_stream(pm_plan plan, int mode, const void* src, void* dst, int64_t nbytes, hipStream_t stream);

/* Kernel timing.  pm_timing_enable(plan, mask) times every launch of the
 * kernel families whose bit (1 << PM_K_*) is set in mask (0 switches timing
 * off); each launch is bracketed by HIP events on the stream it runs on.
 * pm_timing_read(plan, PM_K_*, ...) synchronises that family's events and
 * returns, since the last pm_timing_enable, the summed milliseconds, the
 * number of launches and two byte counts (any output may be NULL):
 *   total_bytes        algorithmic bytes: every array the launch touches
 *                      read or written once, the implementation's own
 *                      intermediates included (sort keys, CIC records,
 *                      particle lists, halo faces, the spectra between the
 *                      passes of a 3-D FFT);
 *   total_method_bytes what the method itself must move: the particle state
 *                      and mesh fields of the operation read or written once,
 *                      each 3-D FFT as one read of its input and one write of
 *                      its output (charged to its first and last pass), no
 *                      intermediates.
 * At most 1024 launches per family are recorded between two reads; launches
 * beyond that are counted and reported as a PM_EINVAL error by the read. */
#define PM_K_BIN         1   /* paint: drift + tile binning                  */
#define PM_K_FFT_R2C_Z   2   /* real-to-complex pass along z                 */
#define PM_K_FFT_C2R_Z   3   /* complex-to-real pass along z                 */
#define PM_K_FFT_LINES   4   /* strided complex passes along y and x         */
#define PM_K_FFT_POISSON 5   /* first inverse pass with the Poisson kernel   */
#define PM_K_GATHER      6   /* tiled CIC gather (+ kick / VJP)              */
#define PM_K_SCATTER     7   /* paint: per-tile particle lists               */
#define PM_K_PAINT_TILES 8   /* paint: LDS tile sums                         */
#define PM_K_HALO        9   /* paint: halo faces into the mesh              */
#define PM_K_LIGHTCONE  10   /* light-cone observation, its VJP and bump      */
int pm_timing_enable(pm_plan plan, unsigned mask);
int pm_timing_read(pm_plan plan, int kernel, double* total_ms, int64_t* launches, double* total_bytes,
                   double* total_method_bytes);

#ifdef __cplusplus
}
#endif
#endif /* PM_H */
