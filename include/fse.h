/*
 * fse.h -- C ABI of the MI355X split-step library for the rotating
 * space-fractional nonlinear Schroedinger / Gross-Pitaevskii equation with a
 * GauSum nonlocal potential.
 *
 * Method (Antoine, Tang, Zhang, arXiv:1512.03210):
 *   i psi_t = [ (1/2)(-Lap + m^2)^s + V + beta|psi|^2 + lambda Phi - Omega Lz ] psi,
 *   Phi = U * |psi|^2                                   (eqs. SFSE, NonLocalPot)
 * solved in rotating Lagrangian coordinates x = A(t) x~ (eqs. Amatrix,
 * transform, FSE1_Rot) by the TS2-GauSum time splitting (eqs. tssp1-tssp3):
 * half a linear step, exact in Fourier space; a full nonlinear step whose
 * density is constant, with the nonlocal potential from the Gaussian-sum
 * method of Section 2; half a linear step.
 *
 * Conventions shared by every call
 * --------------------------------
 * Grid.   d = 2 or 3 axes; axis 0 is the slowest (x~), axis d-1 the
 *         contiguous one.  N[j] points on [-L[j], L[j]), x_l = -L + l h,
 *         h = 2L/N (the periodic endpoint is not stored).  Each N[j] is even,
 *         16 <= N[j] <= 512, and has no prime factor other than 2 and 3.
 * Arrays. psi: C-contiguous [N0][N1]([N2]) interleaved complex, complex128
 *         (FSE_C128) or complex64 (FSE_C64) per the plan's precision; real
 *         arrays (rho, Phi) are double or float in the same layout.  All
 *         array arguments are DEVICE pointers owned by the caller; the
 *         library never frees them.  Scalar outputs are double, written to
 *         DEVICE memory (read them after synchronising the stream).
 * Streams. `stream` is a hipStream_t passed as void* (NULL = default stream).
 *         Calls are asynchronous on that stream; only fse_plan_create and
 *         fse_plan_destroy synchronise.  A plan must not be used from two
 *         host threads at once.
 * Time.   The plan keeps the time t of the state in DEVICE memory (FP64);
 *         the rotating-frame trap W(x~,t) = V(A(t) x~), a dipole axis that
 *         turns in the rotating frame and a turning optical lattice depend on
 *         it.  Kernels read it on the device: fse_step and fse_step4 advance
 *         it on the stream by nsteps*dt, and a call recorded into a HIP graph
 *         (fse_step, fse_step4, fse_energy, fse_moments,
 *         fse_nonlocal_potential, fse_mass, fse_angular_momentum,
 *         fse_step_adjoint) replays at the time the plan has when the replay
 *         runs.  Buffers a call clears are cleared by a kernel, not a runtime
 *         memset.  Before capturing, make one eager call of each kind (first
 *         calls allocate tables and buffers).
 * Errors. Every call returns an fse_status; nothing is thrown across the ABI.
 *         fse_last_error() returns a message for the calling thread's last
 *         failure.
 */
#ifndef FSE_H
#define FSE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fse_plan_s* fse_plan; /* opaque; owned by the library */

typedef enum {
    FSE_OK = 0,
    FSE_ERR_ARG = -1,          /* invalid argument (dimension, size, parameter) */
    FSE_ERR_UNSUPPORTED = -2,  /* valid physics the library does not implement */
    FSE_ERR_NOMEM = -3,        /* device or host allocation failed */
    FSE_ERR_HIP = -4,          /* a HIP runtime call failed */
    FSE_ERR_NUMERIC = -5,      /* non-finite parameter or result */
    FSE_ERR_STATE = -6         /* call not valid in the plan's current state */
} fse_status;
/* A NULL plan or batch handle, or a NULL where a pointer is required, returns
 * FSE_ERR_ARG (message in fse_last_error) before anything touches the device;
 * destroying a NULL handle does nothing and returns FSE_OK. */

typedef enum { FSE_C128 = 0, FSE_C64 = 1 } fse_precision;

/* Nonlocal kernel U (eq. Kernel):
 *   FSE_K_NONE    -- no nonlocal term (lambda is ignored);
 *   FSE_K_COULOMB -- U = prefactor / |x|^mu, 0 < mu <= d-1; the paper's
 *                    Coulomb-type kernel has prefactor 1/(2^{d-1} pi);
 *   FSE_K_DDI3    -- d = 3 dipole-dipole kernel -delta - 3 d_nn (1/(4 pi |x|))
 *                    with unit dipole axis n;
 *   FSE_K_DDI2    -- d = 2 dipole-dipole kernel
 *                    -(3/2)(d_{n_perp n_perp} - n3^2 Lap_perp)(1/(2 pi |x|)),
 *                    n = (n_perp, n3) a unit vector.
 * Any unit axis.  A coordinate axis (3D), or an in-plane part along x or y
 * (2D), gives a multiplier even in every frequency, stored whole.  A tilted
 * axis (products n_i n_j in the symbol), or with Omega != 0 any axis off z,
 * which turns in the rotating Lagrangian coordinates as m(t) = A^{-1}(t) n
 * (eq. Kernel_Rot), is applied as c0 + Khat_C kappa^T M kappa inside the
 * padded convolution, M the time average of m m^T over each nonlinear
 * sub-step (M = n n^T for H psi and the ground state, whose frame has the
 * axis n); its odd products are zero at Nyquist indices.  Such an axis needs
 * the contiguous axis N[d-1] <= 256 and is not taken by the batch. */
typedef enum { FSE_K_NONE = 0, FSE_K_COULOMB = 1, FSE_K_DDI3 = 2, FSE_K_DDI2 = 3 } fse_kernel_kind;

typedef struct {
    int kind;          /* fse_kernel_kind */
    double mu;         /* Coulomb exponent (ignored for the dipoles) */
    double prefactor;  /* c in U = c/|x|^mu (ignored for the dipoles, which use 1/(4 pi), 1/(2 pi)) */
    double n[3];       /* unit dipole axis (DDI3, DDI2) */
    double delta;      /* near-field radius of the GauSum split; <= 0 selects 1e-4 * max L */
    double ht;         /* sinc-quadrature step of the Gaussian sum; <= 0 selects 0.14 */
} fse_kernel;

/* Host-only validation of a problem description; no device work.
 * Returns FSE_OK, FSE_ERR_ARG or FSE_ERR_UNSUPPORTED (message in fse_last_error). */
fse_status fse_plan_check(int d, const int* N, const double* L, double s, double Omega,
                          const double* gamma, double beta, double lambda,
                          const fse_kernel* kernel, int precision);

/* Build a plan for one grid and parameter set (eqs. SFSE, NonLocalPot, harm_poten).
 * gamma[d] are the trap frequencies of V = sum_v gamma_v^2 v^2 / 2; m >= 0 is
 * the mass term of (-Lap + m^2)^s.  Precomputes on the host, in FP64, the
 * GauSum multiplier (Section 2: the Gaussian sum eq. GS-Gene, the tensor
 * eq. tensor, the near-field correction eq. taylor) and the FFT twiddles,
 * and allocates the device workspace.  Synchronises `stream`.
 * The plan's time starts at 0. */
fse_status fse_plan_create(fse_plan* out, int d, const int* N, const double* L, double s,
                           double Omega, const double* gamma, double beta, double lambda,
                           const fse_kernel* kernel, int precision, double m, void* stream);

fse_status fse_plan_destroy(fse_plan plan);

/* Device bytes held by the plan (multiplier, twiddles, workspace). */
fse_status fse_workspace_size(fse_plan plan, size_t* bytes);

/* Bytes of the step's scratch (the padded transform intermediates X1 and, in
 * 3D, X2; 0 without a nonlocal term) that fse_set_workspace can take from the
 * caller. */
fse_status fse_scratch_size(fse_plan plan, size_t* bytes);

/* Use a caller-owned device buffer (e.g. torch-allocated) of at least
 * fse_scratch_size bytes, 256-byte aligned, as the step's scratch; the plan
 * frees its own (synchronising the device).  The contents are not kept across
 * calls, so the caller may reuse the memory between calls on the plan's
 * stream, but must keep it allocated while calls run.  dev_ptr = NULL returns
 * to plan-owned scratch.  FSE_ERR_ARG if too small or misaligned.  If the
 * plan-owned scratch cannot be allocated again (FSE_ERR_NOMEM), the plan has
 * none until a later call succeeds, and calls that need it return
 * FSE_ERR_STATE. */
fse_status fse_set_workspace(fse_plan plan, void* dev_ptr, size_t bytes);

/* Set / read the plan's time (host value, written to / read from the device
 * copy).  Both wait for the device to finish its queued work first (host
 * queries: not for use inside a graph capture).  FSE_ERR_ARG for a
 * non-finite t. */
fse_status fse_set_time(fse_plan plan, double t);
fse_status fse_get_time(fse_plan plan, double* t);

/* nsteps TS2-GauSum steps of size dt (eqs. tssp1-tssp3), in place on psi
 * (rotating Lagrangian coordinates).  Adjacent half linear steps of
 * consecutive steps are merged into one full step, which is exact algebra.
 * dt may be negative (backward in time); nsteps >= 0.  t += nsteps*dt. */
fse_status fse_step(fse_plan plan, void* psi, int nsteps, double dt, void* stream);

/* FP64 mass renormalisation of a step call (fse_step, fse_step4).  The split
 * step conserves the discrete mass exactly (eq. MassEnerg); in FP32 the FFT
 * twiddle tables carry modulus residuals of up to 5e-8 that bias it by about
 * 1e-8 per transform, depending on the data.  With renormalisation on, a call
 * reduces the mass of psi in FP64 at its start, reduces it again before its
 * last pass (the inverse FFT of axis 0) and scales that pass's output by
 * sqrt(M_start / M_before): the call returns a state with the mass it was
 * given (to FP64 reduction accuracy), at the cost of two extra reads of the
 * state per call.  The bias inside a call is not corrected.  Default: on for
 * complex64 plans, off for complex128.  Asynchronous; graph-capturable. */
fse_status fse_set_mass_renorm(fse_plan plan, int enable);

/* Whether it is on, and (factor_mass nullable, 3 doubles) the last call's
 * factor, the mass before the exit pass and the mass at the call's start
 * (synchronises the device). */
fse_status fse_get_mass_renorm(fse_plan plan, int* enabled, double* factor_mass);

/* Optional numeric guard (failure detection; the paper has none).  With
 * tol > 0, every fse_step and fse_step4 call ends with an FP64 mass reduction
 * of its result on the call's stream, compared on the device with the mass
 * at the first guarded call: a non-finite mass or a relative change above tol
 * trips the guard.  The outcome reaches the host behind an event: a later
 * fse_step or fse_step4 call that finds the check completed and tripped
 * returns FSE_ERR_NUMERIC without launching anything, and so does every such
 * call after it until fse_set_guard is called again.  fse_set_guard
 * synchronises the device and resets the reference mass and the flag;
 * tol <= 0 turns the guard off (the default).  Each guarded call reads the
 * state once more and copies 24 bytes to pinned host memory (not meant for
 * graph capture).  FSE_ERR_ARG if tol is not finite. */
fse_status fse_set_guard(fse_plan plan, double tol);

/* Waits for the last guarded call's check.  *tripped = 1 if the guard has
 * tripped; masses (nullable, 2 doubles): the reference mass and the mass of
 * the last completed check (NaN before the first check). */
fse_status fse_guard_status(fse_plan plan, int* tripped, double* masses);

/* nsteps fourth-order steps of size dt, in place on psi: each step is the
 * symmetric triple-jump composition of TS2-GauSum steps of lengths w1 dt,
 * w0 dt, w1 dt, w1 = 1/(2 - 2^{1/3}), w0 = 1 - 2 w1 < 0 (the paper notes
 * that TS2 extends to higher-order splitting, end of Section 4.2; the
 * composition is Yoshida's).  Same state convention, arguments, stream
 * semantics and time update as fse_step; a step costs three nonlinear and
 * three kinetic sub-steps (half linear steps that meet are merged). */
fse_status fse_step4(fse_plan plan, void* psi, int nsteps, double dt, void* stream);

/* Entries of a pass schedule (fse_plan_tune, fse_plan_get_schedule, fse_plan_set_schedule). */
#define FSE_NSCHED 5

/* Autotuner of the plan's pass schedule.  Times, on the plan's own workspace,
 * the compiled alternatives of its tunable passes and keeps the fastest:
 *   sched[0]  radix schedule of the kinetic line transform (0 plain, 1 the
 *             alternative, where the line length has one: 256, 512);
 *   sched[1]  radix schedule of the convolution line transform (same values);
 *   sched[2]  visit order of the kinetic line pass (1: the four lines that
 *             share a table row together; 3D only);
 *   sched[3]  radix plan of the step's column transforms along axis 0 (and
 *             axis 1 in 3D): 0 plain, 1 the alternative where the length has
 *             one (256 as 8.8.4 beside 16.16);
 *   sched[4]  radix plan of the fused complex-to-real + nonlinear phase pass
 *             (axis 0): 0 the default (256: 8.8.4 in FP64, 16.16 in
 *             complex64), 1 the other one, where the length has two (256).
 * Another schedule replaces the current one only when it is at least 1 %
 * faster, so repeated tuning is stable.  Results are cached for the process
 * per device name and architecture, grid, precision and presence of the
 * nonlocal term; with cache_path non-NULL they are also looked up in, and
 * appended to, that text file ("key<TAB>s0 s1 s2 s3 s4" lines), so a cached
 * shape is not timed again.  Candidates are timed on whole steps (two TS2
 * steps on the plan's scratch state, every allowed schedule, interleaved over
 * five rounds), since a pass timed alone can stay in the last-level cache.
 * Synchronous on `stream`; allocates the diagnostics buffer and the step's
 * kinetic tables if absent; overwrites the plan's workspace, not the caller's
 * state; the plan's time is unchanged.
 * Without tuning a plan uses the default schedule {0, 0, 1 in 3D FP64 else 0, 0, 0}. */
fse_status fse_plan_tune(fse_plan plan, const char* cache_path, void* stream);

/* The plan's schedule (sched[FSE_NSCHED], as above) and, if tuned_ms is not
 * NULL, the last measurement: 2^FSE_NSCHED values, the time in ms of one step
 * with schedule {k, c, o, v, f} at index k + 2c + 4o + 8v + 16f (-1 where
 * not measured). */
fse_status fse_plan_get_schedule(fse_plan plan, int* sched, double* tuned_ms);

/* Force a schedule (sched[FSE_NSCHED], entries 0 or 1).  FSE_ERR_UNSUPPORTED
 * for an alternative the plan's lengths do not have, or a mirrored order in 2D. */
fse_status fse_plan_set_schedule(fse_plan plan, const int* sched);

/* Optical lattice added to the harmonic trap: V_L = sum_j v[j] sin^2(k[j] x_j)
 * over the d axes, defined in the frame of eq. SFSE (the form of the paper's
 * second ground-state example).  With Omega != 0 it turns in the rotating
 * Lagrangian coordinates of the step, and each nonlinear sub-step integrates
 * it over time by 8-node Gauss-Legendre quadrature (the trap integral P of a
 * non-harmonic V has no closed form); the energy takes its value at the plan's
 * time, H psi and the ground state take it in the frame of eq. SFSE.  v = NULL
 * removes it.  The first call allocates one real array of N points. */
fse_status fse_set_lattice(fse_plan plan, const double* v, const double* k);

/* Optional real potential U(x~) on the plan's grid, added to the nonlinear
 * phase of fse_step and fse_step4 as dt * U and to the potential energy of
 * fse_energy (eq. SFSE with V + U; U is static in the rotating Lagrangian
 * coordinates x~ of the step).  U: device array [N0][N1]([N2]) of doubles
 * (complex128 plans) or floats (complex64 plans), caller-owned; the plan keeps
 * the pointer, not a copy, so the array must stay valid and unchanged while
 * calls that use it run.  NULL clears it.  fse_apply_H and fse_gs_step add U
 * only when Omega = 0 (with rotation the two frames differ) and return
 * FSE_ERR_UNSUPPORTED otherwise. */
fse_status fse_set_potential(fse_plan plan, const void* U);

/* Adjoint (reverse-mode derivative) of nsteps TS2-GauSum steps of size dt
 * from psi0 at the plan's time t.  The paper gives none: this is the discrete
 * adjoint of fse_step, derived by hand (conjugate kinetic phases, reversed
 * FFT order, the self-adjoint GauSum convolution, the linearised nonlinear
 * phase).  Gradient convention, for a real loss L: g = dL/dRe(psi) +
 * i dL/dIm(psi), so that dL = Re sum conj(g) dpsi.
 *   grad:   on entry dL/dpsi(t + nsteps dt), on exit dL/dpsi0 (in place);
 *   grad_U: NULL, or a real array (plan precision) to which dL/dU is added.
 * psi0 is not modified and must not alias grad; the plan's time is unchanged.
 * The forward states of the segment are recomputed from psi0, so a caller
 * keeps one checkpoint per segment.  The first call, or a longer segment
 * than before, allocates nsteps * N * (complex + real) bytes of workspace
 * (synchronising the device); later calls allocate nothing. */
fse_status fse_step_adjoint(fse_plan plan, const void* psi0, int nsteps, double dt,
                            void* grad, void* grad_U, void* stream);

/* out = Lz psi = -i (x d_y - y d_x) psi with Fourier derivatives (the
 * operator of eq. AME, whose expectation fse_angular_momentum returns).
 * out must not alias psi. */
fse_status fse_apply_Lz(fse_plan plan, const void* psi, void* out, void* stream);

/* Gradient of g <Lz> with respect to psi (torch's convention, as
 * fse_step_adjoint): <Lz> = h^d sum conj(psi) Lz psi with Lz Hermitian, so
 *   out = 2 h^d g Lz psi,
 * g = *g_dev (one double in device memory, e.g. the upstream gradient of a
 * loss; NULL means g = 1).  out must not alias psi. */
fse_status fse_angular_momentum_grad(fse_plan plan, const void* psi, const double* g_dev, void* out, void* stream);

/* H psi in the lab frame (the operator of eq. SFSE; with a frozen density it
 * is the operator A^{BE,n} of Section 3.2 without its I/dt part):
 *   H psi = (1/2)(-Lap+m^2)^s psi + (V + beta rho + lambda Phi[rho]) psi - Omega Lz psi,
 * rho = |psi|^2, or rho_frozen (real array) when it is not NULL.
 * psi and Hpsi must not alias. */
fse_status fse_apply_H(fse_plan plan, const void* psi, void* Hpsi, const void* rho_frozen,
                       void* stream);

/* Phi = U * |psi|^2 on the grid (Section 2; eq. NonLocalPot), written as a
 * real array.  Zero when the plan has no kernel. */
fse_status fse_nonlocal_potential(fse_plan plan, const void* psi, void* Phi, void* stream);

/* Mass h^d sum |psi|^2 (eq. mass) -> out_dev[0]. */
fse_status fse_mass(fse_plan plan, const void* psi, double* out_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the mass of
 * fse_mass, computed by the same kernels, with the per-block partial sums in a
 * fixed 32 KiB device array of the library instead of the plan's buffer.  No
 * allocation of any kind; asynchronous on `stream`; out_dev[0] as fse_mass.
 * The partials need 4 x 1024 doubles for any grid size (a larger need would be
 * refused with FSE_ERR_ARG).  All calls on one device share that device's
 * array: calls that overlap on one device (two streams, two host threads)
 * race and must be ordered by the caller. */
fse_status fse_mass_noalloc(fse_plan plan, const void* psi, double* out_dev, void* stream);

/* Energy parts (eq. energy), in rotating coordinates at the plan's time with
 * W(x~,t) = V(A(t)x~):
 * out_dev[0..5] = E_kin, E_pot, E_int, E_non, E_rot = -Omega <Lz>, E_total.
 * Sums are accumulated in FP64 for both precisions. */
fse_status fse_energy(fse_plan plan, const void* psi, double* out_dev, void* stream);

/* <Lz> = h^d sum psi^* (-i)(x D_y - y D_x) psi (eq. AME) -> out_dev[0]. */
fse_status fse_angular_momentum(fse_plan plan, const void* psi, double* out_dev, void* stream);

/* Mass, centre of mass and condensate widths in the lab frame at the plan's
 * time (eqs. mass, CoM, ConWidth; the width is int v^2 |psi|^2, no square
 * root).  psi is in rotating coordinates x~ and is read through x = A(t) x~,
 * A = [[cos Omega t, sin Omega t], [-sin Omega t, cos Omega t]] on (x, y):
 * out_dev[0..6] = N, x_c, y_c, z_c, delta_x, delta_y, delta_z (z entries 0 in
 * 2D), each h^d times an FP64 sum over the grid.  One pass over psi; no
 * allocation; asynchronous on `stream`.  Shares the plan's reduction scratch
 * with the other diagnostics, so calls on one plan must be ordered on one
 * stream. */
fse_status fse_moments(fse_plan plan, const void* psi, double* out_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Ground state: one step of the gradient flow with discrete normalisation,
 * discretised by the semi-implicit backward Euler method (Section 3.2, eqs.
 * gf-eq2 to gffg33).  With rho^n = |psi|^2 and Phi^n = U * rho^n frozen,
 *   A^{BE,n} phi1 = psi / dt,
 *   A^{BE,n} = I/dt + (1/2)(-Lap+m^2)^s + V + beta rho^n + lambda Phi^n - Omega Lz,
 * is solved in the first preconditioned form of eq. precond_type1,
 *   (I + P_Delta A_TF) phi1 = P_Delta psi / dt,  P_Delta = [I/dt + (1/2)(-Lap+m^2)^s]^{-1},
 * by BiCGStab started from psi, until the relative residual of that system is
 * at most tol or maxit iterations have run; then psi <- phi1 / ||phi1||
 * (discrete norm h^d sum |.|^2).  V is the unrotated trap (the frame in which
 * the energy carries -Omega Lz, as fse_apply_H).  Vectors are kept in the
 * plan's precision; inner products and the Krylov scalars are FP64.
 *
 * The call reads the Krylov scalars back to the host every iteration, so it
 * returns only when the step is complete (it synchronises `stream`).  The
 * first call allocates the solver's vectors (ten complex and two real arrays
 * of the grid's size).
 * dt > 0, tol > 0, maxit >= 1.  Returns FSE_ERR_NUMERIC if the recurrence
 * breaks down (a zero denominator); psi is then left unchanged.
 * ------------------------------------------------------------------------- */
typedef struct {
    int iterations;  /* BiCGStab iterations of this step */
    int converged;   /* 1 if the relative residual reached tol */
    double residual; /* final relative residual of the preconditioned system */
    double diff_inf; /* max |psi^{n+1} - psi^n| over the grid (the paper's stopping quantity) */
} fse_gs_stats;

fse_status fse_gs_step(fse_plan plan, void* psi, double dt, double tol, int maxit, fse_gs_stats* stats,
                       void* stream);

/* Ground state to convergence: fse_gs_step repeated until, after a step,
 *   rule 1: ||psi^n - psi^{n+1}||_inf <= eps_diff * dt  (the stopping rule of
 *           the paper's ground-state computations, Section 3.3), or
 *   rule 2: |E(psi^{n+1}) - E(psi^n)| <= eps_energy,
 * or max_steps steps have run (rule 0).  A rule whose tolerance is <= 0 is not
 * used (rule 1 is tested first).  E is the energy of eq. energy in the frame
 * of eq. SFSE (V unrotated, -Omega <Lz>, a dipole along n), the functional
 * the flow decreases, reduced on the device in FP64.  energy_trace (host
 * memory, nullable, at least max_steps + 1 doubles): E(psi^0), E(psi^1), ...
 * up to the last step.  The energy is computed only when eps_energy > 0 or a
 * trace is requested.  Synchronous, as fse_gs_step; tol and maxit are passed
 * to each step.  FSE_ERR_ARG for dt, tol <= 0, maxit or max_steps < 1, or a
 * non-finite tolerance; FSE_ERR_NUMERIC as fse_gs_step (psi then holds the
 * last completed step). */
typedef struct {
    int steps;             /* gradient-flow steps taken */
    int converged;         /* 1 if a stopping rule held */
    int rule;              /* 1 difference, 2 energy change, 0 none (max_steps) */
    int krylov_iterations; /* BiCGStab iterations over all steps */
    double diff_inf;       /* max |psi^{n+1} - psi^n| of the last step */
    double energy;         /* E of the final state (NaN if the energy was not computed) */
    double energy_change;  /* |E^{n+1} - E^n| of the last step (NaN if not computed) */
    double residual;       /* relative residual of the last step's Krylov solve */
} fse_gs_run_stats;

fse_status fse_gs_run(fse_plan plan, void* psi, double dt, double tol, int maxit, int max_steps, double eps_diff,
                      double eps_energy, double* energy_trace, fse_gs_run_stats* stats, void* stream);

/* Host-only: the GauSum multiplier Khat (before any FFT normalisation) on the
 * non-negative frequency octant, out[(k0*(N1+1)+k1)*(N2+1)+k2] for d = 3
 * (out[k0*(N1+1)+k1] for d = 2), kappa_j = pi k_j / (2 L_j), k_j = 0..N_j.
 * The caller owns `out` (host memory, prod(N_j+1) doubles).  This is the
 * table the plan uploads; it needs no GPU.  A tilted dipole axis has no such
 * table (its multiplier is not even in each frequency): FSE_ERR_UNSUPPORTED. */
fse_status fse_gausum_symbol_host(int d, const int* N, const double* L, const fse_kernel* kernel,
                                  double* out);

/* Copies the plan's multiplier (as fse_gausum_symbol_host lays it out) to
 * host memory; for a tilted or turning dipole axis, its Coulomb part Khat_C.
 * FSE_ERR_STATE if the plan has no kernel. */
fse_status fse_get_symbol(fse_plan plan, double* host_out);

/* ---------------------------------------------------------------------------
 * Batched sweep: many independent 2D instances (each its own grid, s, Omega,
 * trap, interactions and time step), stepped together.
 * ------------------------------------------------------------------------- */
typedef struct {
    int N[2];          /* grid of this instance (same rules as fse_plan_create, d = 2) */
    double L[2];       /* half-widths */
    double s, Omega;   /* fractional order, rotation speed */
    double gamma[2];   /* trap frequencies */
    double beta, lambda;
    double dt;         /* time step of this instance (finite, non-zero) */
    double m;          /* mass term */
    fse_kernel kernel; /* nonlocal kernel (kind FSE_K_NONE for none) */
} fse_instance;

typedef struct fse_batch_s* fse_batch; /* opaque; owned by the library */

/* Build a batch of `count` 2D instances (count >= 1) in one precision.  The
 * states live in one packed device buffer supplied by the caller: instance i
 * occupies elements [offsets[i], offsets[i+1]) (fse_batch_offsets), laid out
 * as [N0][N1].  Instances of equal grid size share their GauSum multiplier.
 * Every instance's time starts at 0.  Synchronises `stream`. */
fse_status fse_batch_create(fse_batch* out, int count, const fse_instance* inst, int precision, void* stream);
fse_status fse_batch_destroy(fse_batch batch);

/* Element offsets of the instances in the packed buffer (count + 1 values,
 * host memory owned by the caller). */
fse_status fse_batch_offsets(fse_batch batch, size_t* offsets);

/* nsteps TS2-GauSum steps of every instance (each with its own dt), in place
 * on the packed buffer.  The pass sequence for a given (nsteps, buffer) is
 * captured once into a HIP graph, one parallel branch per group of equal
 * grid size, and replayed on `stream`; instance times live in device memory
 * and advance by nsteps*dt_i per call. */
fse_status fse_batch_step(fse_batch batch, void* psi_packed, int nsteps, void* stream);

/* Per-instance diagnostics, out_dev[7*i + k] (device memory, count x 7):
 * k = 0 mass, 1..6 = E_kin, E_pot, E_int, E_non, E_rot, E_total (as
 * fse_energy, at the instance's current time). */
fse_status fse_batch_reduce(fse_batch batch, const void* psi_packed, double* out_dev, void* stream);

/* Current time of every instance (host memory, count values). */
fse_status fse_batch_times(fse_batch batch, double* t);

/* The FP64 mass renormalisation of fse_set_mass_renorm for every instance of
 * a batch step call: the call reduces each instance's mass at its start and
 * before its exit pass, which scales the instance by sqrt(M_start /
 * M_before) (eq. MassEnerg: the scheme conserves the discrete mass exactly).
 * Default: on for complex64 batches, off for complex128.  Changing it
 * synchronises the device and drops the captured graphs (the next
 * fse_batch_step records them again). */
fse_status fse_batch_set_mass_renorm(fse_batch batch, int enable);

/* Whether it is on, and (factor_mass nullable, host memory, 3 x count doubles)
 * per instance the last call's factor, the mass before the exit pass and the
 * mass at the call's start (1, 1, 1 before the first renormalising call;
 * synchronises the device). */
fse_status fse_batch_get_mass_renorm(fse_batch batch, int* enabled, double* factor_mass);

/* Per-pass timing for benchmarking.  While enabled, fse_step records a HIP
 * event pair on its stream around every kernel launch.  fse_get_profile
 * synchronises those events, adds the elapsed milliseconds per pass kind
 * into ms[k] and the launch counts into count[k] for k < npass (kinds:
 * FSE_PASS_*), and clears the record. */
enum {
    FSE_PASS_EDGE = 0,      /* entry/exit passes of a call */
    FSE_PASS_R2C = 1,       /* axis-0 inverse, density, padded real-to-complex FFT */
    FSE_PASS_PAD_FWD = 2,   /* 3D: padded forward FFT of axis 1 */
    FSE_PASS_CONV = 3,      /* contiguous axis: padded FFT, GauSum multiplier, inverse */
    FSE_PASS_CROP_INV = 4,  /* 3D: cropped inverse FFT of axis 1 */
    FSE_PASS_C2R_PHASE = 5, /* axis-0 complex-to-real, nonlinear phase, forward FFT */
    FSE_PASS_F1 = 6,        /* 3D: forward FFT of axis 1 */
    FSE_PASS_KIN = 7,       /* contiguous axis: FFT, kinetic phase, inverse */
    FSE_PASS_I1 = 8,        /* 3D: inverse FFT of axis 1 */
    FSE_NPASS = 9
};
fse_status fse_set_profiling(fse_plan plan, int enable);
fse_status fse_get_profile(fse_plan plan, double* ms, int* count, int npass);

/* Streaming device-to-device copy of `bytes` bytes (a multiple of 16, both
 * pointers 16-byte aligned) by a plain vector-load/vector-store kernel.  Used
 * to measure the achievable HBM bandwidth and to calibrate the memory
 * counters against a kernel of known traffic. */
fse_status fse_device_copy(void* dst, const void* src, size_t bytes, void* stream);

/* The same copy with non-temporal loads and stores (streaming past the
 * caches), the reference for buffers far beyond the last-level cache. */
fse_status fse_device_copy_nt(void* dst, const void* src, size_t bytes, void* stream);

/* Message describing the calling thread's last error ("" if none). */
const char* fse_last_error(void);

/* Library version string. */
const char* fse_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FSE_H */
