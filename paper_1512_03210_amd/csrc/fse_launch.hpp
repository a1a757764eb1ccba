// Host-side launchers of the split-step kernels, one explicit instantiation
// per precision (fse_launch_f64.hip, fse_launch_f32.hip).  Every launcher
// maps a runtime FFT length onto the kernel template compiled for it and
// returns the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include "fse_types.hpp"

namespace fse {

// Lengths compiled for the strided passes and the density/potential passes
// of axis 0 (N), and for the contiguous line passes (N and 2N).
bool strided_size_ok(int M);
bool line_size_ok(int M);

template <typename R> struct Launch {
    // Strided length-N FFT over [B0][rows][B2]; mode 0 plain (N -> N rows), 1 zero-padded forward
    // (N -> 2N rows), 2 cropped inverse (2N -> N rows).  twN: length-N twiddles, tw2N: length 2N.
    // scale (mode 0 only): null, or a device factor near 1 applied to the output.
    // cv (mode 0): 1 selects the alternative radix plan of the column transform where the length has one.
    static hipError_t strided(int N, bool inv, int mode, const void* in, void* out, int B0, int B2, const void* twN,
                              const void* tw2N, hipStream_t st, const double* scale = nullptr, int cv = 0);
    // Contiguous line pass on lines of N points; mode 0 padded conv (real multiplier over 2N frequencies),
    // 1 kinetic (complex table), 2 fwd, 3 inv.  var 1 selects the alternative radix schedule (AltRadix) of
    // the conv and kinetic transforms where the length has one, else the plain schedule is used.
    static hipError_t line(int N, int mode, void* data, int nlines, const void* mult, LineIdx li, const void* twN,
                           const void* tw2N, hipStream_t st, int var = 0);
    // Axis-0 density + padded real-to-complex FFT; src 0 pending state, 1 physical psi, 2 real density.
    // Padded convolution along the contiguous axis (length N, padded 2N <= 512) with the
    // quadratic-form dipolar multiplier q over the Coulomb-part table.
    static hipError_t conv_qf(int N, void* data, int nlines, const void* mult, LineIdx li, const void* tw2N,
                              const QForm& q, hipStream_t st);
    static hipError_t r2c(int N0, int src, const void* in, void* X1, int C, const void* twN, const void* tw2N,
                          hipStream_t st, int cv = 0);
    // Axis-0 complex-to-real + nonlinear phase; mode 0 full, 1 phase only, 2 potential output only.
    // fv: the fused kernel's radix plan (FusedPlan; modes 0 and 1, where the length has two).
    static hipError_t c2r_phase(int N0, int mode, const void* X1, void* S, void* Phi, int C, const PhaseArgs& pa,
                                const void* twN, const void* tw2N, hipStream_t st, int fv = 0);
    // Batched 2D pass over `count` equal-size instances (kinds in fse_kernels.hpp).
    static hipError_t batch(int kind, int N0, int N1, void* psi, const BInst* bi, int count, int which, LineIdx li,
                            const void* twN0, const void* tw2N0, const void* twN1, const void* tw2N1,
                            hipStream_t st);
    // Batched FP64 mass of `count` equal-size instances of n points (nblk partial sums each): slot 0
    // stores it as the call's start mass, slot 1 as the mass before the exit pass (times mscale, the
    // pending axis-0 inverse's N0) together with the factor that restores the start mass.
    static hipError_t batch_mass(int slot, long n, double mscale, const void* psi, const BInst* bi, int count,
                                 double* partials, int nblk, hipStream_t st);
    // Even Fourier table on the non-negative octant, omega = (|mu|^2 + m2)^s: kind 0 the phase
    // scale * exp(-i tau omega/2), kind 1 the resolvent scale / (c0 + omega/2), kind 2 scale * omega/2.
    static hipError_t build_kin(void* Q, int T0, int T1, int T2, double dmu0, double dmu1, double dmu2, double s,
                                double m2, int kind, double tau, double c0, double scale, hipStream_t st);
    // W = wa (x^2+y^2) + wz z^2 + wc (x^2-y^2) + ws 2xy; with tp set, wc and ws are gd cos / sin(2 Om *tp).
    static hipError_t red_local(const void* psi, const void* Phi, const void* U, long n, const GridGeom& g, double wa,
                                double wz, double wc, double ws, const double* tp, double Om, double gd,
                                double* partials, int slot0, int nblk, hipStream_t st);
    static hipError_t red_kin(const void* ph, long n, const GridGeom& g, double dmu0, double dmu1, double dmu2,
                              double s, double m2, double* partials, int slot0, int nblk, hipStream_t st);
    static hipError_t red_lz(const void* psi, const void* D, long n, const GridGeom& g, int coord_axis,
                             double* partials, int slot0, int nblk, hipStream_t st);
    static hipError_t red_moments(const void* psi, long n, const GridGeom& g, double* partials, int nblk,
                                  hipStream_t st);
    // (what 0 and 1: Omega times *wscale when wscale is not null)
    static hipError_t H_accum(void* H, const void* D, const void* psi, const void* rho_in, const void* Phi,
                              const void* U, long n, const GridGeom& g, int what, double Omega, double beta,
                              double lam, double g0, double g1, double g2, hipStream_t st,
                              const double* wscale = nullptr);
    // Fourier derivative along one axis in one pass, out = D in (out of place allowed): strided axis of
    // [B0][N][B2] (line = false) or nlines = B0 contiguous lines of N points (line = true); the
    // multiplier is i p dmu scale for frequency index p (Nyquist kept as -N/2).
    static hipError_t deriv(int N, bool line, const void* in, void* out, int B0, int B2, const void* twN,
                            double dmu, double scale, hipStream_t st);
    // Ground-state step (kernels in fse_gs.hpp).
    static hipError_t gs_frozen(const void* psi, const void* Phi, const void* U, void* W, long n, const GridGeom& g,
                                double beta, double lam, double g0, double g1, double g2, hipStream_t st);
    // Lattice potential / its time integral into out (k_lattice).
    static hipError_t lattice(void* out, const void* U, long n, const GridGeom& g, const LatArgs& la, hipStream_t st);
    // Adjoint of the split step (kernels in fse_adjoint.hpp).
    static hipError_t adj_theta(const void* psi1, const void* Phi, const void* U, void* theta, void* psi2, long n,
                                const GridGeom& g, const PhaseArgs& pa, hipStream_t st);
    static hipError_t adj_q(const void* g2, const void* psi1, const void* theta, void* q, void* gU, long n,
                            double udt, hipStream_t st);
    static hipError_t adj_g1(void* g, const void* psi1, const void* theta, const void* q, const void* Phiq, long n,
                             double bdt, double ldt, hipStream_t st);
    // First (op 1: pointwise operator + forward FFT of axis 0) and last (op 2: inverse FFT of
    // axis 0 + v) passes of the preconditioned ground-state operator (k_gs_cols).
    static hipError_t gs_cols(int op, int N0, const void* v, const void* Dx, const void* Dy, const void* W,
                              const void* A, void* out, int C, const GridGeom& g, double Omega, const void* twN,
                              hipStream_t st);
    static hipError_t gs_axpy(const void* a, const void* b, void* out, long n, double cr, double ci, hipStream_t st);
    static hipError_t gs_update_xr(void* x, void* r, const void* p, const void* s, const void* t, long n, double ar,
                                   double ai, double wr, double wi, hipStream_t st);
    static hipError_t gs_update_p(void* p, const void* r, const void* v, long n, double br, double bi, double wr,
                                  double wi, hipStream_t st);
    static hipError_t gs_dots(const void* a0, const void* b0, const void* a1, const void* b1, const void* a2,
                              const void* b2, int npair, long n, double* partials, int nblk, hipStream_t st);
    static hipError_t gs_finish(const void* x, void* psi, long n, double scale, double* partials, int nblk,
                                hipStream_t st);
};

// out[k] = sum (op 0) or max (op 1) over the nblk partials of slot k, k < nslot.
hipError_t launch_gs_slots(const double* partials, int nblk, int nslot, int op, double* out, hipStream_t st);

hipError_t launch_batch_time(const BInst* bi, int count, int nsteps, hipStream_t st);
// Per instance (one block each) of the batched mass: see Launch<R>::batch_mass.
hipError_t launch_b_mass_final(const double* partials, int nblk, const BInst* bi, int count, double mscale, int slot,
                               hipStream_t st);

hipError_t launch_copy16(void* dst, const void* src, long n16, hipStream_t st, bool nontemporal = false);

// Whether the line transform of length n has an alternative radix schedule (AltRadix).
bool line_has_alt(int n);
// Whether the column transform of length n has an alternative radix plan (ColPlanOf).
bool col_has_alt(int n);
// Whether the fused complex-to-real + phase kernel of axis length n has a second radix plan (FusedPlan).
bool fused_has_alt(int n);

hipError_t launch_red_final(const double* partials, int nblk, int nslot, int kind, double vol, double n,
                            double beta, double lam, double Omega, double* out, hipStream_t st);

// Zero fill of `bytes` (a multiple of 8) at p, as a kernel: unlike a runtime
// memset it may be recorded into a captured graph like the other passes.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
// Numeric guard: g = {M0, M, flag}.  M0 = M if M0 is NaN (first check); flag
// = 1 if M or M0 is not finite or |M - M0| > tol |M0| (the flag stays set).
hipError_t launch_guard(double* g, double tol, hipStream_t st);
// out[0..6] = lab-frame {N, x_c, y_c, z_c, delta_x, delta_y, delta_z} from
// the eight moment slots; (c, s) = (cos, sin) of the frame angle, or with tp
// set those of Om * *tp.
hipError_t launch_moments_final(const double* partials, int nblk, double vol, double c, double s, const double* tp,
                                double Om, double* out, hipStream_t st);
// r[1] = sqrt(r[0] / (mscale * vol * sum of the nblk partials)) (1 if not finite), r[2] = that mass.
hipError_t launch_renorm_factor(const double* partials, int nblk, double vol, double mscale, double* r,
                                hipStream_t st);
// *t += dtot on the stream (a plan's device time).
hipError_t launch_time_add(double* t, double dtot, hipStream_t st);

}  // namespace fse
