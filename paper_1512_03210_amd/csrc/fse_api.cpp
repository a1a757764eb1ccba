// C ABI of the split-step library: validation, plan set-up and the pass
// schedules of fse_step, fse_nonlocal_potential, fse_apply_H and the
// diagnostics.
//
// Pass schedule of fse_step (rotating Lagrangian coordinates, TS2-GauSum,
// eqs. tssp1-tssp3, with adjacent half linear steps merged).  Between steps
// the state S is psi with every axis in physical space except axis 0, whose
// inverse FFT is still pending:
//   entry:  F0, [F1], line(F_last * kin(dt/2) * I_last), [I1]          -> S
//   step:   r2c      I0(S) -> psi -> rho -> padded R2C along axis 0 -> X1
//           3D:  F1 padded (X1 -> X2), line conv (X2), I1 cropped (X2 -> X1)
//           2D:  line conv (X1)
//           c2r_phase  C2R along axis 0 -> Phi; I0(S) -> psi;
//                      psi *= exp(-i[dt beta rho + lam dt Phi + P]); F0 -> S
//           [F1], line(F_last * kin(dt, or dt/2 after the last step) * I_last), [I1]
//   exit:   I0                                                     -> psi
// ([..] = 3D only.)  The kinetic table carries 1/prod(N_j), the GauSum
// multiplier 1/prod(2 N_j); every FFT is unnormalised.
//
// fse_step_adjoint over a segment of K steps from a checkpoint:
//   forward  psi1_0 = K(dt/2) psi0; per step: Phi[|psi1_k|^2] (r2c, conv,
//            C2R), theta_k and psi2 (pointwise), psi1_{k+1} = K(dt) psi2;
//            psi1_k and theta_k are kept for the whole segment
//   reverse  g = K(-dt/2) g; per step, last to first: q (pointwise, dL/dU),
//            Phi[q] (r2c of a real array, conv, C2R), g1 (pointwise),
//            g = K(-dt) g1 (K(-dt/2) after the first step)
// where K(tau) is a full kinetic pass: F0, [F1], line(F_last * kin * I_last),
// [I1], I0.
#include "../../include/fse.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <array>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fse_host.hpp"
#include "fse_launch.hpp"

namespace {

thread_local std::string g_err;

fse_status fail(fse_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kRedBlocks = 1024;
constexpr int kBatchRed = 32;  // partial sums per instance of the batched mass reduction
constexpr int kRedSlots = 8;
constexpr int kNSched = FSE_NSCHED;  // entries of a pass schedule (fse.h)
constexpr double kTuneMargin = 0.01;  // another schedule must be 1 % faster to replace the current one

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(FSE_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

bool factors_23(int n) {
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

}  // namespace

struct fse_plan_s {
    int d = 0;
    int N[3] = {1, 1, 1};
    double L[3] = {1, 1, 1}, h[3] = {1, 1, 1};
    double s = 1, Omega = 0, gamma[3] = {0, 0, 0}, beta = 0, lambda = 0, m = 0;
    fse_kernel kernel{};
    int prec = FSE_C128;
    bool nl = false;  // nonlocal term present
    double* tdev = nullptr;  // the time t of the state, in device memory (a batch points it into its own array)
    // FP64 mass renormalisation of a step call (fse_set_mass_renorm; on by default for complex64):
    // renorm = {mass at the call's start, factor, mass before the exit pass}, device memory
    bool renorm_on = false;
    double* renorm = nullptr;
    long n = 0;       // grid points
    int C0 = 0;       // columns of the axis-0 passes (n / N0)
    size_t csize = 16, rsize = 8;
    std::map<int, void*> tw;  // device twiddles exp(-2 pi i m/M), by M
    void* khat = nullptr;
    std::vector<double> khat_host;
    void* X1 = nullptr;
    void* X2 = nullptr;
    bool ext_ws = false;  // X1 and X2 live in a caller's buffer (fse_set_workspace)
    // optional optical lattice (fse_set_lattice) and a real n-array for its phase / values
    bool lat = false;
    double lat_v[3] = {0, 0, 0}, lat_k[3] = {0, 0, 0};
    void* lat_buf = nullptr;
    void* kin[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    double kin_tau[7] = {NAN, NAN, NAN, NAN, NAN, NAN, NAN};
    void* diag = nullptr;  // 2 n complex + n real, allocated on first use
    const void* U = nullptr;  // optional caller-owned real potential on the grid (fse_set_potential)
    void* adj = nullptr;      // adjoint workspace (fse_step_adjoint), grown on demand
    // pass schedule: [0] radix variant of the kinetic line transforms, [1] of
    // the convolution line transforms, [2] kinetic visit order (1 mirrored,
    // 3D only), [3] radix plan of the step's column transforms (1: the
    // alternative where the length has one); defaults set at creation,
    // changed by fse_plan_tune/set_schedule
    int sched[kNSched] = {0, 0, 0, 0, 0};
    // dipole with products n_i n_j or an axis that turns in the rotating frame:
    // khat holds the Coulomb-part symbol and each convolution gets a QForm
    bool qf = false;
    double khat_scale = 1.0;  // 1 / prod(2 N_j), carried by khat
    double tune_ms[1 << kNSched] = {};  // ms per step of each schedule, last fse_plan_tune (-1: not timed)
    size_t adj_bytes = 0;
    void* gs = nullptr;    // ground-state solver: 10 n complex + 2 n real, allocated on first use
    double* gs_out = nullptr;
    void* pd = nullptr;    // P_Delta table (layout of the kinetic tables) for pd_c0 = 1/dt
    double pd_c0 = NAN;
    void* ks = nullptr;    // kinetic symbol omega/2 / n (layout of the kinetic tables), built on first use
    double* partials = nullptr;
    // numeric guard (fse_set_guard): guard_dev = {M0 (NaN until the first
    // check), M of the last check, tripped flag}; guard_host is its pinned
    // copy, read only once guard_ev has completed
    double guard_tol = 0.0;
    double* guard_dev = nullptr;
    double* guard_host = nullptr;
    hipEvent_t guard_ev = nullptr;
    bool guard_pending = false, guard_tripped = false;
    size_t bytes = 0;
    std::vector<void*> allocs;
    // profiling: event pairs recorded around launches, by pass kind
    bool prof = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    size_t ev_used = 0;

    int last() const { return N[d - 1]; }
    long lines_last() const { return n / N[d - 1]; }
};

namespace {

void dev_free(fse_plan p, void* ptr, size_t bytes) {
    (void)hipFree(ptr);
    p->allocs.erase(std::remove(p->allocs.begin(), p->allocs.end(), ptr), p->allocs.end());
    p->bytes -= bytes;
}

fse_status dev_alloc(fse_plan p, void** ptr, size_t bytes) {
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) return fail(FSE_ERR_NOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    p->allocs.push_back(*ptr);
    p->bytes += bytes;
    return FSE_OK;
}

// Whether a dipolar kernel needs the quadratic-form multiplier: an axis with a
// product n_i n_j that enters the symbol (its multiplier is not even in each
// frequency alone), or an axis that turns in the rotating frame (Omega != 0,
// n_perp != 0).
bool dipole_needs_form(const fse_kernel* k, double Omega) {
    if (!k || (k->kind != FSE_K_DDI3 && k->kind != FSE_K_DDI2)) return false;
    const double* n = k->n;
    const int nz = (n[0] != 0.0) + (n[1] != 0.0) + (k->kind == FSE_K_DDI3 && n[2] != 0.0);
    return nz > 1 || (Omega != 0.0 && (n[0] != 0.0 || n[1] != 0.0));
}

fse_status check_args(int d, const int* N, const double* L, double s, double Omega, const double* gamma, double beta,
                      double lambda, const fse_kernel* kernel, int precision) {
    if (d != 2 && d != 3) return fail(FSE_ERR_ARG, "d must be 2 or 3 (got %d)", d);
    if (!N || !L || !gamma) return fail(FSE_ERR_ARG, "N, L and gamma must not be NULL");
    const int nmax = (d == 3) ? 256 : 512;
    for (int j = 0; j < d; ++j) {
        if (N[j] < 16 || N[j] > nmax || (N[j] % 2) != 0 || !factors_23(N[j]))
            return fail(FSE_ERR_ARG, "N[%d] = %d: need an even size in [16, %d] with prime factors 2 and 3 only", j,
                        N[j], nmax);
        if (!fse::strided_size_ok(N[j]))
            return fail(FSE_ERR_UNSUPPORTED, "N[%d] = %d has no compiled FFT length", j, N[j]);
        if (!(L[j] > 0.0) || !std::isfinite(L[j])) return fail(FSE_ERR_ARG, "L[%d] must be finite and > 0", j);
        if (!std::isfinite(gamma[j])) return fail(FSE_ERR_ARG, "gamma[%d] must be finite", j);
    }
    if (!(s > 0.0) || !std::isfinite(s)) return fail(FSE_ERR_ARG, "s must be finite and > 0");
    if (!std::isfinite(Omega) || !std::isfinite(beta) || !std::isfinite(lambda))
        return fail(FSE_ERR_ARG, "Omega, beta and lambda must be finite");
    if (precision != FSE_C128 && precision != FSE_C64) return fail(FSE_ERR_ARG, "unknown precision %d", precision);
    if (kernel) {
        if (kernel->kind == FSE_K_COULOMB) {
            if (!(kernel->mu > 0.0) || kernel->mu > d - 1 + 1e-15)
                return fail(FSE_ERR_ARG, "Coulomb exponent mu must lie in (0, d-1]");
            if (!std::isfinite(kernel->prefactor)) return fail(FSE_ERR_ARG, "kernel prefactor must be finite");
        } else if (kernel->kind == FSE_K_DDI3 || kernel->kind == FSE_K_DDI2) {
            const bool three = kernel->kind == FSE_K_DDI3;
            if (d != (three ? 3 : 2))
                return fail(FSE_ERR_ARG, "the %dD dipolar kernel needs d = %d", three ? 3 : 2, three ? 3 : 2);
            const double* n = kernel->n;
            if (!std::isfinite(n[0]) || !std::isfinite(n[1]) || !std::isfinite(n[2]))
                return fail(FSE_ERR_ARG, "dipole axis must be finite");
            const double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
            if (std::fabs(nn - 1.0) > 1e-12) return fail(FSE_ERR_ARG, "dipole axis must be a unit vector");
            // A tilted or turning axis applies its quadratic form inside the
            // one-pass padded convolution, which needs a padded length 2N <= 512.
            if (dipole_needs_form(kernel, Omega) && 2 * N[d - 1] > 512)
                return fail(FSE_ERR_UNSUPPORTED,
                            "a tilted or turning dipole axis needs N[%d] <= 256 (padded convolution in one pass)", d - 1);
        } else if (kernel->kind != FSE_K_NONE) {
            return fail(FSE_ERR_ARG, "unknown kernel kind %d", kernel->kind);
        }
        if (!std::isfinite(kernel->delta) || !std::isfinite(kernel->ht))
            return fail(FSE_ERR_ARG, "kernel delta and ht must be finite");
    }
    // 3D: the padded transform of axis 1 runs at length 2 N1 (at most 512 since N <= 256).
    if (kernel && kernel->kind != FSE_K_NONE && d == 3 && !fse::strided_size_ok(2 * N[1]))
        return fail(FSE_ERR_UNSUPPORTED, "padded length %d has no compiled FFT length", 2 * N[1]);
    return FSE_OK;
}

// Nearest representable (cos, sin) for FP64.  For FP32, of the four pairs
// that bracket the exact values, the one whose squared modulus is closest to 1:
// every transform reuses the table, so a magnitude bias would accumulate in the
// mass of the complex64 state (about 3x less drift over 1000 steps).
template <typename T> std::vector<T> twiddles(int M) {
    using F = decltype(T{}.x);
    std::vector<T> v(M);
    for (int k = 0; k < M; ++k) {
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)M;
        const long double cx = cosl(a), cy = sinl(a);
        v[k].x = (F)cx;
        v[k].y = (F)cy;
        if (sizeof(F) == 4) {
            const F xs[2] = {v[k].x, ((long double)v[k].x < cx) ? std::nextafter(v[k].x, F(2)) : std::nextafter(v[k].x, F(-2))};
            const F ys[2] = {v[k].y, ((long double)v[k].y < cy) ? std::nextafter(v[k].y, F(2)) : std::nextafter(v[k].y, F(-2))};
            long double best = 1.0L;
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    const long double e = fabsl((long double)xs[i] * xs[i] + (long double)ys[j] * ys[j] - 1.0L);
                    if (e < best) {
                        best = e;
                        v[k].x = xs[i];
                        v[k].y = ys[j];
                    }
                }
        }
    }
    return v;
}

fse_status upload_twiddles(fse_plan p, int M) {
    if (p->tw.count(M)) return FSE_OK;
    void* ptr = nullptr;
    fse_status st = dev_alloc(p, &ptr, (size_t)M * p->csize);
    if (st != FSE_OK) return st;
    if (p->prec == FSE_C128) {
        auto v = twiddles<double2>(M);
        HIPCHK(hipMemcpy(ptr, v.data(), (size_t)M * sizeof(double2), hipMemcpyHostToDevice));
    } else {
        auto v = twiddles<float2>(M);
        HIPCHK(hipMemcpy(ptr, v.data(), (size_t)M * sizeof(float2), hipMemcpyHostToDevice));
    }
    p->tw[M] = ptr;
    return FSE_OK;
}

// Record the start event of a launch of pass kind k (no-op unless profiling).
fse_status prof_begin(fse_plan p, int k, hipStream_t st) {
    if (!p->prof) return FSE_OK;
    if (p->ev_used + 2 > p->ev.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            p->ev.push_back(e);
        }
        p->ev_kind.resize(p->ev.size() / 2);
    }
    p->ev_kind[p->ev_used / 2] = k;
    HIPCHK(hipEventRecord(p->ev[p->ev_used], st));
    return FSE_OK;
}

fse_status prof_end(fse_plan p, hipStream_t st) {
    if (!p->prof) return FSE_OK;
    HIPCHK(hipEventRecord(p->ev[p->ev_used + 1], st));
    p->ev_used += 2;
    return FSE_OK;
}

// Launch wrapped in profiling events.
#define PLAUNCH(p, kind, st, expr)                     \
    do {                                               \
        fse_status ps_ = prof_begin((p), (kind), (st)); \
        if (ps_ != FSE_OK) return ps_;                 \
        HIPCHK(expr);                                  \
        ps_ = prof_end((p), (st));                     \
        if (ps_ != FSE_OK) return ps_;                 \
    } while (0)

fse::GridGeom geom(const fse_plan p) {
    fse::GridGeom g;
    g.d = p->d;
    g.N0 = p->N[0];
    g.N1 = p->N[1];
    g.N2 = (p->d == 3) ? p->N[2] : 1;
    g.x0 = -p->L[0];
    g.hx = p->h[0];
    g.y0 = -p->L[1];
    g.hy = p->h[1];
    g.z0 = (p->d == 3) ? -p->L[2] : 0.0;
    g.hz = (p->d == 3) ? p->h[2] : 0.0;
    return g;
}

double dmu(const fse_plan p, int j) { return (j < p->d) ? 2.0 * kPi / (2.0 * p->L[j]) : 0.0; }

// Kinetic table for step length tau; slot 0 holds the half step at the ends
// of a call, slot 1 the merged halves between steps, slot 2 the merged halves
// between the sub-steps of a composed step, slots 3-6 the adjoint's +dt/2,
// +dt, -dt/2, -dt; each is rebuilt only when its tau changes.
template <typename R> fse_status kin_table(fse_plan p, double tau, int slot, void** out, hipStream_t st) {
    if (p->kin[slot] && p->kin_tau[slot] == tau) {
        *out = p->kin[slot];
        return FSE_OK;
    }
    const int T0 = p->N[0] / 2 + 1, T1 = (p->d == 3) ? p->N[1] / 2 + 1 : 1;
    const int T2 = p->last() / 2 + 1;
    const double dm1 = (p->d == 3) ? dmu(p, 1) : 0.0;
    const double dm2 = dmu(p, p->d - 1);
    if (!p->kin[slot]) {
        fse_status s = dev_alloc(p, &p->kin[slot], (size_t)T0 * T1 * T2 * p->csize);
        if (s != FSE_OK) return s;
    }
    HIPCHK(fse::Launch<R>::build_kin(p->kin[slot], T0, T1, T2, dmu(p, 0), dm1, dm2, p->s, p->m * p->m, 0, tau, 0.0,
                                     1.0 / (double)p->n, st));
    p->kin_tau[slot] = tau;
    *out = p->kin[slot];
    return FSE_OK;
}

fse::LineIdx kin_index(const fse_plan p) {
    fse::LineIdx li;
    if (p->d == 3) {
        li.D1 = p->N[1];
        li.F0 = p->N[0];
        li.F1 = p->N[1];
        li.T1 = p->N[1] / 2 + 1;
        li.T2 = p->N[2] / 2 + 1;
        // the four lines (+-k0, +-k1) share a table row: visited together when
        // the schedule says so
        li.X0 = li.X1 = p->sched[2];
    } else {
        li.D1 = 1;
        li.F0 = p->N[0];
        li.F1 = 0;
        li.T1 = 1;
        li.T2 = p->N[1] / 2 + 1;
    }
    return li;
}

fse::LineIdx conv_index(const fse_plan p) {
    fse::LineIdx li;
    if (p->d == 3) {
        li.D1 = 2 * p->N[1];
        li.F0 = 0;
        li.F1 = 2 * p->N[1];
        li.T1 = p->N[1] + 1;
        li.T2 = p->N[2] + 1;
        // lines k1 and 2 N1 - k1 share a multiplier row: visited side by side
        // (one workgroup), the row is fetched once
        li.X1 = 1;
    } else {
        li.D1 = 1;
        li.F0 = 0;
        li.F1 = 0;
        li.T1 = 1;
        li.T2 = p->N[1] + 1;
    }
    return li;
}

// A time for the time-dependent coefficients: the plan's device time plus an
// offset known on the host (dev), or a fixed time (not dev; t = 0 is the frame
// of eq. SFSE, where H psi and the ground state live).
struct TimeRef {
    bool dev;
    double off;
};
constexpr TimeRef kFrame{false, 0.0};
TimeRef at_plan(double off = 0.0) { return TimeRef{true, off}; }

double gdiff(const fse_plan p) { return (p->gamma[0] * p->gamma[0] - p->gamma[1] * p->gamma[1]) / 4.0; }

// Whether the rotating part of the trap depends on time (rotation and gx != gy).
bool trap_turns(const fse_plan p) { return p->Omega != 0.0 && gdiff(p) != 0.0; }

fse::PhaseArgs phase_args(const fse_plan p, TimeRef tn, double dt) {
    fse::PhaseArgs a;
    a.x0 = -p->L[0];
    a.hx = p->h[0];
    a.y0 = -p->L[1];
    a.hy = p->h[1];
    a.z0 = (p->d == 3) ? -p->L[2] : 0.0;
    a.hz = (p->d == 3) ? p->h[2] : 0.0;
    a.N2 = (p->d == 3) ? p->N[2] : 0;
    const double gx2 = p->gamma[0] * p->gamma[0], gy2 = p->gamma[1] * p->gamma[1];
    const double gz2 = (p->d == 3) ? p->gamma[2] * p->gamma[2] : 0.0;
    a.ca = dt * (gx2 + gy2) / 4.0;
    a.cz = dt * gz2 / 2.0;
    if (tn.dev && trap_turns(p)) {  // evaluated by the kernel at the device time
        a.tp = p->tdev;
        a.toff = tn.off;
        a.tau = dt;
        a.Om = p->Omega;
        a.gd = gdiff(p);
        a.sf = std::sin(p->Omega * dt) / p->Omega;
        a.cc = a.cs = 0.0;
    } else {  // independent of the time, or at a fixed time
        fse::trap_rotating(tn.off, dt, p->Omega, gdiff(p), &a.cc, &a.cs);
    }
    a.bdt = p->beta * dt;
    a.ldt = p->lambda * dt;
    a.U = p->U;
    a.udt = dt;
    return a;
}

// The dipolar multiplier of a qf plan over [t, t+tau] in the rotating
// Lagrangian coordinates (tau = 0: at the instant t; t = 0 is also the frame of
// H psi and of the ground state, where the axis is n): the axis
// m(s) = A(s)^{-1} n is n_perp turned by +Omega s, and the time average of
// m m^T has, for each harmonic cos/sin(a + b s), its midpoint value times
// sinc(b tau / 2) (eq. Kernel_Rot).
fse::QForm qform(const fse_plan p, TimeRef t, double tau) {
    const double* n = p->kernel.n;
    fse::QForm q{};
    q.r = std::hypot(n[0], n[1]);
    q.phi0 = (q.r > 0.0) ? std::atan2(n[1], n[0]) : 0.0;
    q.n2 = n[2];
    q.Om = p->Omega;
    q.kscale = p->khat_scale;
    q.d3 = (p->d == 3) ? 1 : 0;
    q.dk0 = kPi / (2.0 * p->L[0]);
    q.n0 = p->N[0];
    if (p->d == 3) {
        q.dk1 = kPi / (2.0 * p->L[1]);
        q.dk2 = kPi / (2.0 * p->L[2]);
        q.n1 = p->N[1];
    } else {
        q.dk1 = 0.0;
        q.dk2 = kPi / (2.0 * p->L[1]);
        q.n1 = 0;
    }
    if (t.dev && p->Omega != 0.0) {  // a turning axis: averaged on the device at the plan's time
        q.tp = p->tdev;
        q.toff = t.off;
        q.tau = tau;
    }
    fse::qform_fill(q, t.dev ? 0.0 : t.off, tau);  // (time-independent without rotation)
    return q;
}

// Padded convolution along the contiguous axis with the plan's multiplier; a
// qf plan uses the quadratic form over [t, t+tau].
template <typename R> hipError_t conv_line(fse_plan p, TimeRef t, double tau, hipStream_t st) {
    using L = fse::Launch<R>;
    const int NL = p->last();
    void* X = (p->d == 3) ? p->X2 : p->X1;
    const int nl = (p->d == 3) ? (p->N[0] + 1) * 2 * p->N[1] : p->N[0] + 1;
    if (p->qf) return L::conv_qf(NL, X, nl, p->khat, conv_index(p), p->tw[2 * NL], qform(p, t, tau), st);
    return L::line(NL, 0, X, nl, p->khat, conv_index(p), p->tw[NL], p->tw[2 * NL], st, p->sched[1]);
}

// Lattice arguments: its time integral over [t, t+tau] in rotating coordinates
// (8-node Gauss-Legendre in time; the trap integral P of a non-harmonic V has
// no closed form), plus tau U; or its value at the instant t (tau = 0), plus U.
fse::LatArgs lat_args(const fse_plan p, TimeRef t, double tau) {
    fse::LatArgs la{};
    for (int j = 0; j < 3; ++j) {
        la.v[j] = p->lat_v[j];
        la.k[j] = p->lat_k[j];
    }
    la.tau = tau;
    la.Om = p->Omega;
    if (tau == 0.0) {
        la.nq = 1;
        la.gx[0] = 0.0;
        la.gw[0] = 2.0;
        la.uf = 1.0;
    } else {
        std::vector<double> x, w;
        fse::gauss_legendre(8, x, w);
        la.nq = 8;
        for (int q = 0; q < 8; ++q) {
            la.gx[q] = x[q];
            la.gw[q] = w[q];
        }
        la.uf = tau;
    }
    if (t.dev && p->Omega != 0.0) {  // the lattice turns: nodes at the device time
        la.tp = p->tdev;
        la.toff = t.off;
    }
    fse::lat_fill(la, t.dev ? 0.0 : t.off);  // (time-independent without rotation)
    return la;
}

// The potential array the pointwise kernels add: the grid potential U, or with a
// lattice the lattice in the frame at time t (frame = true: the frame of
// eq. SFSE, for H psi and the ground state) plus U, written to lat_buf.
template <typename R> const void* extra_potential(fse_plan p, TimeRef t, hipStream_t st, hipError_t* e) {
    *e = hipSuccess;
    if (!p->lat) return p->U;
    const fse::LatArgs la = lat_args(p, t, 0.0);
    *e = fse::Launch<R>::lattice(p->lat_buf, p->U, p->n, geom(p), la, st);
    return p->lat_buf;
}

// Whether the nonlocal scratch (X1, and X2 in 3D) is in place: an allocation
// that failed in fse_set_workspace leaves the plan without it until a later
// call succeeds, and no kernel may then be launched on it.
fse_status scratch_ready(const fse_plan p) {
    if (p->nl && (!p->X1 || (p->d == 3 && !p->X2)))
        return fail(FSE_ERR_STATE, "the plan has no scratch (fse_set_workspace failed to allocate it)");
    return FSE_OK;
}

// Zero-padded GauSum convolution of the density held in X1 (after r2c), result back in X1.
template <typename R> fse_status conv_passes(fse_plan p, TimeRef t, double tau, hipStream_t st) {
    using L = fse::Launch<R>;
    if (fse_status s = scratch_ready(p); s != FSE_OK) return s;
    if (p->d == 3) {
        const int N1 = p->N[1], N2 = p->N[2];
        HIPCHK(L::strided(N1, false, 1, p->X1, p->X2, p->N[0] + 1, N2, p->tw[N1], p->tw[2 * N1], st));
        HIPCHK(conv_line<R>(p, t, tau, st));
        HIPCHK(L::strided(N1, true, 2, p->X2, p->X1, p->N[0] + 1, N2, p->tw[N1], p->tw[2 * N1], st));
    } else {
        HIPCHK(conv_line<R>(p, t, tau, st));
    }
    return FSE_OK;
}

// Phi[rho] into a real array; src 1: rho = |psi|^2, 2: rho given.
// (t, tau: the time and averaging interval of a turning dipole axis, see qform)
template <typename R>
fse_status potential_impl(fse_plan p, const void* src, int srckind, void* Phi, TimeRef t, double tau, hipStream_t st) {
    using L = fse::Launch<R>;
    if (!p->nl) {
        HIPCHK(fse::launch_zero(Phi, (size_t)p->n * p->rsize, st));
        return FSE_OK;
    }
    const int N0 = p->N[0];
    if (fse_status s = scratch_ready(p); s != FSE_OK) return s;
    HIPCHK(L::r2c(N0, srckind, src, p->X1, p->C0, p->tw[N0], p->tw[2 * N0], st));
    fse_status s = conv_passes<R>(p, t, tau, st);
    if (s != FSE_OK) return s;
    fse::PhaseArgs pa = phase_args(p, kFrame, 0.0);  // (mode 2 writes the potential only)
    HIPCHK(L::c2r_phase(N0, 2, p->X1, nullptr, Phi, p->C0, pa, p->tw[N0], p->tw[2 * N0], st));
    return FSE_OK;
}

fse_status ensure_diag(fse_plan p) {
    if (p->diag) return FSE_OK;
    return dev_alloc(p, &p->diag, (size_t)p->n * (2 * p->csize + p->rsize));
}

// One call advances nsteps steps.  A step is a composition of TS2 sub-steps
// of lengths w_j dt: the Strang step itself (order 2), or the symmetric
// triple jump w = (w1, 1 - 2 w1, w1), w1 = 1/(2 - 2^{1/3}) (order 4).  The
// half linear steps that meet between sub-steps are merged into one kinetic
// pass of length (w_j + w_{j+1}) dt / 2.
template <typename R>
fse_status step_impl(fse_plan p, void* psi, int nsteps, double dt, int order, hipStream_t st) {
    using L = fse::Launch<R>;
    if (fse_status s = scratch_ready(p); s != FSE_OK) return s;
    double w[3] = {1.0, 0.0, 0.0};
    int nw = 1;
    if (order == 4) {
        const double w1 = 1.0 / (2.0 - std::cbrt(2.0));
        w[0] = w[2] = w1;
        w[1] = 1.0 - 2.0 * w1;
        nw = 3;
    }
    void *kh = nullptr, *kf = nullptr, *ki_tab = nullptr;
    fse_status s = kin_table<R>(p, 0.5 * w[0] * dt, 0, &kh, st);
    if (s != FSE_OK) return s;
    if (nsteps > 1) {
        s = kin_table<R>(p, 0.5 * (w[nw - 1] + w[0]) * dt, 1, &kf, st);
        if (s != FSE_OK) return s;
    }
    if (nw > 1) {  // symmetric weights: every inner junction has the same length
        s = kin_table<R>(p, 0.5 * (w[0] + w[1]) * dt, 2, &ki_tab, st);
        if (s != FSE_OK) return s;
    }
    const int N0 = p->N[0];
    const int NL = p->last();
    const int nlines = (int)p->lines_last();
    const fse::LineIdx ki = kin_index(p);
    const int N1 = p->N[1], N2 = (p->d == 3) ? p->N[2] : 1;
    const double vol = p->h[0] * p->h[1] * ((p->d == 3) ? p->h[2] : 1.0);
    if (p->renorm_on) {  // the mass at the start of the call, FP64
        PLAUNCH(p, FSE_PASS_EDGE, st,
                L::red_local(psi, nullptr, nullptr, p->n, geom(p), 0, 0, 0, 0, nullptr, 0, 0, p->partials, 0,
                             kRedBlocks, st));
        PLAUNCH(p, FSE_PASS_EDGE, st,
                fse::launch_red_final(p->partials, kRedBlocks, 1, 0, vol, (double)p->n, 0, 0, 0, p->renorm, st));
    }
    // entry: half linear step, leaving the axis-0 inverse pending
    const int cv = p->sched[3];
    PLAUNCH(p, FSE_PASS_EDGE, st, L::strided(N0, false, 0, psi, psi, 1, p->C0, p->tw[N0], nullptr, st, nullptr, cv));
    if (p->d == 3)
        PLAUNCH(p, FSE_PASS_EDGE, st,
                L::strided(N1, false, 0, psi, psi, N0, N2, p->tw[N1], nullptr, st, nullptr, cv));
    PLAUNCH(p, FSE_PASS_EDGE, st, L::line(NL, 1, psi, nlines, kh, ki, p->tw[NL], nullptr, st, p->sched[0]));
    if (p->d == 3)
        PLAUNCH(p, FSE_PASS_EDGE, st, L::strided(N1, true, 0, psi, psi, N0, N2, p->tw[N1], nullptr, st, nullptr, cv));
    for (int k = 0; k < nsteps; ++k) {
        double tj = k * dt;  // offset of the sub-step from the plan's time at the call
        for (int j = 0; j < nw; ++j) {
            const double tau = w[j] * dt;
            fse::PhaseArgs pa = phase_args(p, at_plan(tj), tau);
            if (p->lat) {
                // the sub-step's lattice integral (and tau U) as the phase's grid potential
                HIPCHK(L::lattice(p->lat_buf, p->U, p->n, geom(p), lat_args(p, at_plan(tj), tau), st));
                pa.U = p->lat_buf;
                pa.udt = 1.0;
            }
            tj += tau;
            if (p->nl) {
                PLAUNCH(p, FSE_PASS_R2C, st, L::r2c(N0, 0, psi, p->X1, p->C0, p->tw[N0], p->tw[2 * N0], st, cv));
                if (p->d == 3) {
                    PLAUNCH(p, FSE_PASS_PAD_FWD, st,
                            L::strided(N1, false, 1, p->X1, p->X2, N0 + 1, N2, p->tw[N1], p->tw[2 * N1], st));
                    PLAUNCH(p, FSE_PASS_CONV, st, conv_line<R>(p, at_plan(tj - tau), tau, st));
                    PLAUNCH(p, FSE_PASS_CROP_INV, st,
                            L::strided(N1, true, 2, p->X2, p->X1, N0 + 1, N2, p->tw[N1], p->tw[2 * N1], st));
                } else {
                    PLAUNCH(p, FSE_PASS_CONV, st, conv_line<R>(p, at_plan(tj - tau), tau, st));
                }
                PLAUNCH(p, FSE_PASS_C2R_PHASE, st,
                        L::c2r_phase(N0, 0, p->X1, psi, nullptr, p->C0, pa, p->tw[N0], p->tw[2 * N0], st,
                                     p->sched[4]));
            } else {
                PLAUNCH(p, FSE_PASS_C2R_PHASE, st,
                        L::c2r_phase(N0, 1, nullptr, psi, nullptr, p->C0, pa, p->tw[N0], p->tw[2 * N0], st,
                                     p->sched[4]));
            }
            void* tab = (j < nw - 1) ? ki_tab : (k == nsteps - 1) ? kh : kf;
            if (p->d == 3)
                PLAUNCH(p, FSE_PASS_F1, st,
                        L::strided(N1, false, 0, psi, psi, N0, N2, p->tw[N1], nullptr, st, nullptr, cv));
            PLAUNCH(p, FSE_PASS_KIN, st, L::line(NL, 1, psi, nlines, tab, ki, p->tw[NL], nullptr, st, p->sched[0]));
            if (p->d == 3)
                PLAUNCH(p, FSE_PASS_I1, st,
                        L::strided(N1, true, 0, psi, psi, N0, N2, p->tw[N1], nullptr, st, nullptr, cv));
        }
    }
    const double* scale = nullptr;
    if (p->renorm_on) {
        // mass of the state before the exit pass (the pending axis-0 inverse scales it by N0), and the factor
        // that restores the mass at the start of the call, applied by the exit pass
        PLAUNCH(p, FSE_PASS_EDGE, st,
                L::red_local(psi, nullptr, nullptr, p->n, geom(p), 0, 0, 0, 0, nullptr, 0, 0, p->partials, 0,
                             kRedBlocks, st));
        PLAUNCH(p, FSE_PASS_EDGE, st, fse::launch_renorm_factor(p->partials, kRedBlocks, vol, (double)N0, p->renorm, st));
        scale = p->renorm + 1;
    }
    PLAUNCH(p, FSE_PASS_EDGE, st, L::strided(N0, true, 0, psi, psi, 1, p->C0, p->tw[N0], nullptr, st, scale, cv));
    HIPCHK(fse::launch_time_add(p->tdev, nsteps * dt, st));
    return FSE_OK;
}

// Energy / mass / Lz reductions; kind 0 mass, 1 energy, 2 Lz.
template <typename R> hipError_t deriv_axis(fse_plan p, int axis, const void* v, void* out, hipStream_t st);

// tr: the time of W(x~, t) and of a turning dipole axis (the plan's device time, or kFrame for the frame of
// eq. SFSE, where the ground state is sought).
template <typename R>
fse_status reduce_impl(fse_plan p, const void* psi, int kind, double* out, hipStream_t st, TimeRef tr = at_plan()) {
    using L = fse::Launch<R>;
    const fse::GridGeom g = geom(p);
    const double vol = p->h[0] * p->h[1] * ((p->d == 3) ? p->h[2] : 1.0);
    if (kind == 0) {
        HIPCHK(L::red_local(psi, nullptr, nullptr, p->n, g, 0, 0, 0, 0, nullptr, 0, 0, p->partials, 0, kRedBlocks, st));
        HIPCHK(fse::launch_red_final(p->partials, kRedBlocks, 1, 0, vol, (double)p->n, p->beta, p->lambda, p->Omega,
                                     out, st));
        return FSE_OK;
    }
    fse_status s = ensure_diag(p);
    if (s != FSE_OK) return s;
    char* base = static_cast<char*>(p->diag);
    void* A = base;
    void* B = base + (size_t)p->n * p->csize;
    void* Phi = base + (size_t)p->n * 2 * p->csize;
    int nslot = 7;
    if (kind == 1) {
        const bool use_phi = p->nl;
        if (use_phi) {
            s = potential_impl<R>(p, psi, 1, Phi, tr, 0.0, st);
            if (s != FSE_OK) return s;
        }
        const double gx2 = p->gamma[0] * p->gamma[0], gy2 = p->gamma[1] * p->gamma[1];
        const double gz2 = (p->d == 3) ? p->gamma[2] * p->gamma[2] : 0.0;
        hipError_t ee;
        const void* Ux = extra_potential<R>(p, tr, st, &ee);
        HIPCHK(ee);
        // W(x~, t) = V(A(t) x~): its rotating part at the device time, or at a fixed time
        const bool dev = tr.dev && trap_turns(p);
        const double th = 2.0 * p->Omega * tr.off;
        HIPCHK(L::red_local(psi, use_phi ? Phi : nullptr, Ux, p->n, g, (gx2 + gy2) / 4.0, gz2 / 2.0,
                            dev ? 0.0 : gdiff(p) * std::cos(th), dev ? 0.0 : gdiff(p) * std::sin(th),
                            dev ? p->tdev : nullptr, p->Omega, gdiff(p), p->partials, 0, kRedBlocks, st));
    } else {
        // slots 0..4 unused for Lz; keep them defined
        HIPCHK(fse::launch_zero(p->partials, sizeof(double) * kRedBlocks * 5, st));
    }
    if (kind == 1) {
        // kinetic energy by Parseval from the spectrum (first pass out of place)
        const int N0 = p->N[0];
        HIPCHK(L::strided(N0, false, 0, psi, A, 1, p->C0, p->tw[N0], nullptr, st));
        if (p->d == 3) HIPCHK(L::strided(p->N[1], false, 0, A, A, N0, p->N[2], p->tw[p->N[1]], nullptr, st));
        HIPCHK(L::line(p->last(), 2, A, (int)p->lines_last(), nullptr, fse::LineIdx{1, 0, 0, 1, 1},
                       p->tw[p->last()], nullptr, st));
        HIPCHK(L::red_kin(A, p->n, g, dmu(p, 0), dmu(p, 1), dmu(p, 2), p->s, p->m * p->m, p->partials, 4, kRedBlocks,
                          st));
    }
    // D_y psi against x, D_x psi against y (one derivative pass each)
    for (int pass = 0; pass < 2; ++pass) {
        HIPCHK(deriv_axis<R>(p, pass == 0 ? 1 : 0, psi, B, st));
        HIPCHK(L::red_lz(psi, B, p->n, g, pass == 0 ? 0 : 1, p->partials, 5 + pass, kRedBlocks, st));
    }
    HIPCHK(fse::launch_red_final(p->partials, kRedBlocks, nslot, kind, vol, (double)p->n, p->beta, p->lambda, p->Omega,
                                 out, st));
    return FSE_OK;
}

// Kinetic flow over all axes, dst = K src with K = exp(-i tau omega/2) (tab
// built for tau): physical space in and out, out of place allowed.
template <typename R> fse_status kin_full(fse_plan p, const void* src, void* dst, void* tab, hipStream_t st) {
    using L = fse::Launch<R>;
    const int N0 = p->N[0], NL = p->last();
    HIPCHK(L::strided(N0, false, 0, src, dst, 1, p->C0, p->tw[N0], nullptr, st));
    if (p->d == 3) HIPCHK(L::strided(p->N[1], false, 0, dst, dst, N0, p->N[2], p->tw[p->N[1]], nullptr, st));
    HIPCHK(L::line(NL, 1, dst, (int)p->lines_last(), tab, kin_index(p), p->tw[NL], nullptr, st, p->sched[0]));
    if (p->d == 3) HIPCHK(L::strided(p->N[1], true, 0, dst, dst, N0, p->N[2], p->tw[p->N[1]], nullptr, st));
    HIPCHK(L::strided(N0, true, 0, dst, dst, 1, p->C0, p->tw[N0], nullptr, st));
    return FSE_OK;
}

// Adjoint workspace: the state psi1 = K(dt/2) psi of every step of a segment
// (complex), its phase theta (real), and two real arrays (q, Phi).
fse_status ensure_adj(fse_plan p, int nsteps) {
    const size_t need = (size_t)nsteps * p->n * (p->csize + p->rsize) + 2 * (size_t)p->n * p->rsize;
    if (p->adj && p->adj_bytes >= need) return FSE_OK;
    if (p->adj) {
        dev_free(p, p->adj, p->adj_bytes);
        p->adj = nullptr;
        p->adj_bytes = 0;
    }
    fse_status s = dev_alloc(p, &p->adj, need);
    if (s != FSE_OK) return s;
    p->adj_bytes = need;
    return FSE_OK;
}

// Reverse of nsteps TS2 steps from psi0 at the plan's time: g holds dL/dpsi at
// the end of the segment on entry and dL/dpsi0 on exit; gU (optional) gains
// dL/dU.  The forward states of the segment are recomputed first (the caller
// keeps checkpoints), then the steps are reversed with the kinetic halves that
// meet merged into one pass of -dt.
template <typename R>
fse_status adjoint_impl(fse_plan p, const void* psi0, int nsteps, double dt, void* g, void* gU, hipStream_t st) {
    using L = fse::Launch<R>;
    fse_status s = ensure_adj(p, nsteps);
    if (s != FSE_OK) return s;
    void *kp_h = nullptr, *kp_f = nullptr, *km_h = nullptr, *km_f = nullptr;
    if ((s = kin_table<R>(p, 0.5 * dt, 3, &kp_h, st)) != FSE_OK) return s;
    if ((s = kin_table<R>(p, -0.5 * dt, 5, &km_h, st)) != FSE_OK) return s;
    if (nsteps > 1) {
        if ((s = kin_table<R>(p, dt, 4, &kp_f, st)) != FSE_OK) return s;
        if ((s = kin_table<R>(p, -dt, 6, &km_f, st)) != FSE_OK) return s;
    }
    const size_t cb = (size_t)p->n * p->csize, rb = (size_t)p->n * p->rsize;
    char* base = static_cast<char*>(p->adj);
    char* thb = base + (size_t)nsteps * cb;
    auto S = [&](int k) { return static_cast<void*>(base + (size_t)k * cb); };
    auto TH = [&](int k) { return static_cast<void*>(thb + (size_t)k * rb); };
    void* q = thb + (size_t)nsteps * rb;
    void* Phi = thb + (size_t)(nsteps + 1) * rb;
    const fse::GridGeom gg = geom(p);
    // forward: psi1 and theta of every step
    if ((s = kin_full<R>(p, psi0, S(0), kp_h, st)) != FSE_OK) return s;
    for (int k = 0; k < nsteps; ++k) {
        if (p->nl && (s = potential_impl<R>(p, S(k), 1, Phi, at_plan(k * dt), dt, st)) != FSE_OK) return s;
        fse::PhaseArgs pa = phase_args(p, at_plan(k * dt), dt);
        const void* Ux = p->U;
        if (p->lat) {
            HIPCHK(L::lattice(p->lat_buf, p->U, p->n, gg, lat_args(p, at_plan(k * dt), dt), st));
            Ux = p->lat_buf;
            pa.udt = 1.0;
        }
        void* next = (k + 1 < nsteps) ? S(k + 1) : nullptr;
        HIPCHK(L::adj_theta(S(k), p->nl ? Phi : nullptr, Ux, TH(k), next, p->n, gg, pa, st));
        if (next && (s = kin_full<R>(p, next, next, kp_f, st)) != FSE_OK) return s;
    }
    // reverse
    if ((s = kin_full<R>(p, g, g, km_h, st)) != FSE_OK) return s;
    for (int k = nsteps - 1; k >= 0; --k) {
        HIPCHK(L::adj_q(g, S(k), TH(k), q, gU, p->n, dt, st));
        if (p->nl && (s = potential_impl<R>(p, q, 2, Phi, at_plan(k * dt), dt, st)) != FSE_OK) return s;
        HIPCHK(L::adj_g1(g, S(k), TH(k), q, p->nl ? Phi : nullptr, p->n, p->beta * dt, p->lambda * dt, st));
        if ((s = kin_full<R>(p, g, g, (k > 0) ? km_f : km_h, st)) != FSE_OK) return s;
    }
    return FSE_OK;
}

// out = c Lz psi = -i c (x D_y - y D_x) psi, c = scale (times *gdev when gdev is not null).
template <typename R>
fse_status apply_Lz_impl(fse_plan p, const void* psi, void* out, hipStream_t st, double scale = 1.0,
                         const double* gdev = nullptr) {
    using L = fse::Launch<R>;
    fse_status s = ensure_diag(p);
    if (s != FSE_OK) return s;
    void* B = static_cast<char*>(p->diag) + (size_t)p->n * p->csize;
    const fse::GridGeom g = geom(p);
    HIPCHK(fse::launch_zero(out, (size_t)p->n * p->csize, st));
    HIPCHK(deriv_axis<R>(p, 1, psi, B, st));
    HIPCHK(L::H_accum(out, B, psi, nullptr, nullptr, nullptr, p->n, g, 0, -scale, 0, 0, 0, 0, 0, st, gdev));
    HIPCHK(deriv_axis<R>(p, 0, psi, B, st));
    HIPCHK(L::H_accum(out, B, psi, nullptr, nullptr, nullptr, p->n, g, 1, -scale, 0, 0, 0, 0, 0, st, gdev));
    return FSE_OK;
}

// ---------------------------------------------------------------------------
// Autotuner.  Candidates: the radix schedule of the kinetic line transform
// (plain or alternative), the radix schedule of the convolution line
// transform, the kinetic visit order (3D: plain or mirrored), the radix plan
// of the column transforms and that of the fused phase pass (where the
// lengths have two).  Every combination is timed on whole steps over the
// plan's scratch state (the data does not change the work; timing single
// passes instead misleads where a repeated pass stays in the last-level
// cache), and another schedule replaces the current one only if it is 1 %
// faster, so that repeated tuning gives the same schedule.  Choices are cached
// per device name, architecture, grid, precision and kernel presence for the
// process, and optionally in a text file of "key<TAB>k c o v f" lines.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, std::array<int, kNSched>> g_tune_cache;

// Numeric guard.  guard_poll: the outcome of the last completed check, without
// waiting (a check still running is looked at by a later call).  guard_check:
// after a step call, the mass of the result against the reference, on the
// stream, and a copy of the outcome to pinned memory behind guard_ev.
fse_status guard_poll(fse_plan p) {
    if (p->guard_pending && hipEventQuery(p->guard_ev) == hipSuccess) {
        p->guard_pending = false;
        if (p->guard_host[2] != 0.0) p->guard_tripped = true;
    }
    if (p->guard_tripped)
        return fail(FSE_ERR_NUMERIC,
                    "numeric guard: mass %.17g against %.17g at the first guarded call (relative tolerance %g); "
                    "fse_set_guard resets it",
                    p->guard_host[1], p->guard_host[0], p->guard_tol);
    return FSE_OK;
}

fse_status guard_check(fse_plan p, const void* psi, hipStream_t st) {
    if (p->guard_tol <= 0.0) return FSE_OK;
    fse_status s = (p->prec == FSE_C128) ? reduce_impl<double>(p, psi, 0, p->guard_dev + 1, st)
                                         : reduce_impl<float>(p, psi, 0, p->guard_dev + 1, st);
    if (s != FSE_OK) return s;
    HIPCHK(fse::launch_guard(p->guard_dev, p->guard_tol, st));
    HIPCHK(hipMemcpyAsync(p->guard_host, p->guard_dev, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(p->guard_ev, st));
    p->guard_pending = true;
    return FSE_OK;
}

std::string tune_key(const fse_plan p) {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
    char buf[512];
    snprintf(buf, sizeof(buf), "%s|%s|d%d|%dx%dx%d|%s|%s", prop.name, prop.gcnArchName, p->d, p->N[0], p->N[1],
             (p->d == 3) ? p->N[2] : 1, p->prec == FSE_C128 ? "c128" : "c64", p->nl ? "conv" : "local");
    for (char* c = buf; *c; ++c)
        if (*c == '\t' || *c == '\n') *c = ' ';
    return std::string(buf);
}

// Times the candidates fs[c] (each one launch): after two warm-up launches of
// each, five rounds in which every candidate runs ten launches back to back;
// ms[c] is the best round's average (rounds interleave the candidates, so
// slow drifts of clock or temperature affect them alike).
fse_status time_candidates(const std::vector<std::function<hipError_t()>>& fs, hipStream_t st, double* ms) {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(FSE_ERR_HIP, "hipEventCreate failed");
    }
    fse_status s = FSE_OK;
    for (size_t c = 0; c < fs.size(); ++c) ms[c] = 1e30;
    for (int round = -1; round < 5 && s == FSE_OK; ++round) {
        for (size_t c = 0; c < fs.size() && s == FSE_OK; ++c) {
            const int reps = (round < 0) ? 2 : 10;
            if (hipEventRecord(e0, st) != hipSuccess) s = fail(FSE_ERR_HIP, "hipEventRecord failed");
            for (int k = 0; k < reps && s == FSE_OK; ++k) {
                const hipError_t e = fs[c]();
                if (e != hipSuccess) s = fail(FSE_ERR_HIP, "tuning launch failed: %s", hipGetErrorString(e));
            }
            if (s == FSE_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                s = fail(FSE_ERR_HIP, "event wait failed");
            float t = 0.0f;
            if (s == FSE_OK && round >= 0 && hipEventElapsedTime(&t, e0, e1) == hipSuccess)
                ms[c] = std::min(ms[c], (double)t / reps);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}

// The plan's device time, read or written after the device has drained (host queries, not for capture).
fse_status read_time(const fse_plan p, double* t) {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(t, p->tdev, sizeof(double), hipMemcpyDeviceToHost));
    return FSE_OK;
}

fse_status write_time(fse_plan p, double t) {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(p->tdev, &t, sizeof(double), hipMemcpyHostToDevice));
    return FSE_OK;
}

bool kin_has_alt(const fse_plan p) { return fse::line_has_alt(p->last()); }
// The step's column transforms run along axis 0 (and axis 1 in 3D).
bool cols_have_alt(const fse_plan p) {
    return fse::col_has_alt(p->N[0]) || (p->d == 3 && fse::col_has_alt(p->N[1]));
}
bool fused_has_alt(const fse_plan p) { return fse::fused_has_alt(p->N[0]); }
bool conv_has_alt(const fse_plan p) {
    const int n = p->last();
    return p->nl && ((2 * n <= 512) ? fse::line_has_alt(2 * n) : fse::line_has_alt(n));
}

// Times every schedule the plan allows on whole steps (two TS2 steps on the
// plan's scratch state, so that each pass meets the caches as in a run) and
// keeps the fastest; tune_ms[k + 2c + 4o + 8v + 16f] is the time per step of
// schedule {k, c, o, v, f}.  The plan's time is restored.
template <typename R> fse_status tune_measure(fse_plan p, hipStream_t st) {
    fse_status s = ensure_diag(p);
    if (s != FSE_OK) return s;
    void* A = p->diag;
    HIPCHK(fse::launch_zero(A, (size_t)p->n * p->csize, st));
    const double dt = std::isnan(p->kin_tau[1]) ? 1e-3 : p->kin_tau[1];
    double t_keep = 0.0;
    if ((s = read_time(p, &t_keep)) != FSE_OK) return s;
    const bool prof_keep = p->prof;
    p->prof = false;
    int keep[kNSched];
    for (int q = 0; q < kNSched; ++q) keep[q] = p->sched[q];
    for (double& t : p->tune_ms) t = -1.0;
    std::vector<std::array<int, kNSched>> cands;
    for (int f = 0; f < (fused_has_alt(p) ? 2 : 1); ++f)
        for (int v = 0; v < (cols_have_alt(p) ? 2 : 1); ++v)
            for (int o = 0; o < ((p->d == 3) ? 2 : 1); ++o)
                for (int c = 0; c < (conv_has_alt(p) ? 2 : 1); ++c)
                    for (int k = 0; k < (kin_has_alt(p) ? 2 : 1); ++k) cands.push_back({k, c, o, v, f});
    std::vector<std::function<hipError_t()>> fs;
    for (const auto& cd : cands)
        fs.push_back([=]() {
            for (int q = 0; q < kNSched; ++q) p->sched[q] = cd[q];
            return step_impl<R>(p, A, 2, dt, 2, st) == FSE_OK ? hipSuccess : hipErrorLaunchFailure;
        });
    std::vector<double> ms(fs.size());
    s = time_candidates(fs, st, ms.data());
    p->prof = prof_keep;
    for (int q = 0; q < kNSched; ++q) p->sched[q] = keep[q];
    if (s != FSE_OK) return s;
    if ((s = write_time(p, t_keep)) != FSE_OK) return s;
    int best = -1;
    double tbest = 0.0;
    for (size_t c = 0; c < cands.size(); ++c) {
        const auto& cd = cands[c];
        p->tune_ms[cd[0] + 2 * cd[1] + 4 * cd[2] + 8 * cd[3] + 16 * cd[4]] = 0.5 * ms[c];
        if (std::equal(cd.begin(), cd.end(), keep)) {
            best = (int)c;
            tbest = ms[c];
        }
    }
    // keep the current schedule unless another one is faster by more than the
    // threshold (repeated tuning then returns the same schedule)
    for (size_t c = 0; c < cands.size(); ++c)
        if (ms[c] < (1.0 - kTuneMargin) * tbest) {
            tbest = ms[c];
            best = (int)c;
        }
    for (int q = 0; q < kNSched; ++q) p->sched[q] = cands[best][q];
    return FSE_OK;
}

// Lab-frame mass, centre of mass and widths: one moment pass, then the
// rotation x = A(t) x~ applied to the FP64 totals.
template <typename R> fse_status moments_impl(fse_plan p, const void* psi, double* out, hipStream_t st) {
    const double vol = p->h[0] * p->h[1] * ((p->d == 3) ? p->h[2] : 1.0);
    HIPCHK(fse::Launch<R>::red_moments(psi, p->n, geom(p), p->partials, kRedBlocks, st));
    // the frame angle Omega t at the device time
    HIPCHK(fse::launch_moments_final(p->partials, kRedBlocks, vol, 1.0, 0.0, p->Omega != 0.0 ? p->tdev : nullptr,
                                     p->Omega, out, st));
    return FSE_OK;
}

template <typename R> fse_status apply_H_impl(fse_plan p, const void* psi, void* H, const void* rho, hipStream_t st) {
    using L = fse::Launch<R>;
    fse_status s = ensure_diag(p);
    if (s != FSE_OK) return s;
    const fse::GridGeom g = geom(p);
    char* base = static_cast<char*>(p->diag);
    void* B = base + (size_t)p->n * p->csize;
    void* Phi = base + (size_t)p->n * 2 * p->csize;
    if (p->nl) {
        s = potential_impl<R>(p, rho ? rho : psi, rho ? 2 : 1, Phi, kFrame, 0.0, st);
        if (s != FSE_OK) return s;
    }
    // kinetic part: H = (1/2)(-Lap+m^2)^s psi through the strided forward passes
    // (the first out of place), one line pass (FFT, times omega/2 / n,
    // inverse) and the strided inverse passes
    const int T0 = p->N[0] / 2 + 1, T1 = (p->d == 3) ? p->N[1] / 2 + 1 : 1, T2 = p->last() / 2 + 1;
    if (!p->ks) {
        if ((s = dev_alloc(p, &p->ks, (size_t)T0 * T1 * T2 * p->csize)) != FSE_OK) return s;
        HIPCHK(L::build_kin(p->ks, T0, T1, T2, dmu(p, 0), (p->d == 3) ? dmu(p, 1) : 0.0, dmu(p, p->d - 1), p->s,
                            p->m * p->m, 2, 0.0, 0.0, 1.0 / (double)p->n, st));
    }
    const int N0 = p->N[0], NL = p->last();
    HIPCHK(L::strided(N0, false, 0, psi, H, 1, p->C0, p->tw[N0], nullptr, st));
    if (p->d == 3) HIPCHK(L::strided(p->N[1], false, 0, H, H, N0, p->N[2], p->tw[p->N[1]], nullptr, st));
    HIPCHK(L::line(NL, 1, H, (int)p->lines_last(), p->ks, kin_index(p), p->tw[NL], nullptr, st, p->sched[0]));
    if (p->d == 3) HIPCHK(L::strided(p->N[1], true, 0, H, H, N0, p->N[2], p->tw[p->N[1]], nullptr, st));
    HIPCHK(L::strided(N0, true, 0, H, H, 1, p->C0, p->tw[N0], nullptr, st));
    if (p->Omega != 0.0) {
        // -Omega Lz psi = i Omega (x D_y psi - y D_x psi), one derivative pass per axis
        HIPCHK(deriv_axis<R>(p, 1, psi, B, st));
        HIPCHK(L::H_accum(H, B, psi, nullptr, nullptr, nullptr, p->n, g, 0, p->Omega, 0, 0, 0, 0, 0, st));
        HIPCHK(deriv_axis<R>(p, 0, psi, B, st));
        HIPCHK(L::H_accum(H, B, psi, nullptr, nullptr, nullptr, p->n, g, 1, p->Omega, 0, 0, 0, 0, 0, st));
    }
    hipError_t ee;
    const void* Ux = extra_potential<R>(p, kFrame, st, &ee);
    HIPCHK(ee);
    HIPCHK(L::H_accum(H, nullptr, psi, rho, p->nl ? Phi : nullptr, Ux, p->n, g, 2, p->Omega, p->beta, p->lambda,
                      p->gamma[0], p->gamma[1], (p->d == 3) ? p->gamma[2] : 0.0, st));
    return FSE_OK;
}

// ---------------------------------------------------------------------------
// Ground-state step (Section 3.2): backward-Euler GFDN, first preconditioned
// system of eq. precond_type1, BiCGStab with FP64 scalars.
// ---------------------------------------------------------------------------
struct GsBuf {
    void *x, *r, *r0, *pv, *v, *sv, *t, *A, *Dx, *Dy;  // complex, n each
    void *W, *Phi;                                     // real, n each
};

fse_status ensure_gs(fse_plan p, GsBuf* b) {
    if (!p->gs) {
        fse_status st = dev_alloc(p, &p->gs, (size_t)p->n * (10 * p->csize + 2 * p->rsize));
        if (st != FSE_OK) return st;
        st = dev_alloc(p, (void**)&p->gs_out, sizeof(double) * 8);
        if (st != FSE_OK) return st;
    }
    char* c = static_cast<char*>(p->gs);
    void** v[10] = {&b->x, &b->r, &b->r0, &b->pv, &b->v, &b->sv, &b->t, &b->A, &b->Dx, &b->Dy};
    for (int k = 0; k < 10; ++k) *v[k] = c + (size_t)k * p->n * p->csize;
    b->W = c + (size_t)10 * p->n * p->csize;
    b->Phi = c + (size_t)10 * p->n * p->csize + (size_t)p->n * p->rsize;
    return FSE_OK;
}

// The P_Delta table [c0 + omega/2]^{-1} / n on the kinetic tables' octant,
// rebuilt when c0 = 1/dt changes.
template <typename R> fse_status pd_table(fse_plan p, double c0, hipStream_t st) {
    if (p->pd && p->pd_c0 == c0) return FSE_OK;
    const int T0 = p->N[0] / 2 + 1, T1 = (p->d == 3) ? p->N[1] / 2 + 1 : 1;
    const int T2 = p->last() / 2 + 1;
    if (!p->pd) {
        fse_status s = dev_alloc(p, &p->pd, (size_t)T0 * T1 * T2 * p->csize);
        if (s != FSE_OK) return s;
    }
    HIPCHK(fse::Launch<R>::build_kin(p->pd, T0, T1, T2, dmu(p, 0), (p->d == 3) ? dmu(p, 1) : 0.0,
                                     dmu(p, p->d - 1), p->s, p->m * p->m, 1, 0.0, c0, 1.0 / (double)p->n, st));
    p->pd_c0 = c0;
    return FSE_OK;
}

// a <- P_Delta a: the strided forward passes, one line pass (forward FFT of
// the contiguous axis, times the table, inverse), the strided inverse passes.
template <typename R> fse_status pd_apply(fse_plan p, void* a, hipStream_t st) {
    using L = fse::Launch<R>;
    const int N0 = p->N[0], NL = p->last();
    HIPCHK(L::strided(N0, false, 0, a, a, 1, p->C0, p->tw[N0], nullptr, st));
    if (p->d == 3) HIPCHK(L::strided(p->N[1], false, 0, a, a, N0, p->N[2], p->tw[p->N[1]], nullptr, st));
    HIPCHK(L::line(NL, 1, a, (int)p->lines_last(), p->pd, kin_index(p), p->tw[NL], nullptr, st, p->sched[0]));
    if (p->d == 3) HIPCHK(L::strided(p->N[1], true, 0, a, a, N0, p->N[2], p->tw[p->N[1]], nullptr, st));
    HIPCHK(L::strided(N0, true, 0, a, a, 1, p->C0, p->tw[N0], nullptr, st));
    return FSE_OK;
}

// out = D_axis v (axis 0 or 1) in one pass: only the transform along that axis
// is needed, the multiplier depends on nothing else.
template <typename R> hipError_t deriv_axis(fse_plan p, int axis, const void* v, void* out, hipStream_t st) {
    using L = fse::Launch<R>;
    const int Na = p->N[axis];
    const double sc = 1.0 / (double)Na;
    if (axis == 0) return L::deriv(Na, false, v, out, 1, p->C0, p->tw[Na], dmu(p, 0), sc, st);
    if (p->d == 3) return L::deriv(Na, false, v, out, p->N[0], p->N[2], p->tw[Na], dmu(p, 1), sc, st);
    return L::deriv(Na, true, v, out, p->N[0], 0, p->tw[Na], dmu(p, 1), sc, st);
}

// out = v + P_Delta (W v - Omega Lz v) (P_Delta's table is current).
template <typename R> fse_status gs_apply_M(fse_plan p, const GsBuf& b, const void* v, void* out, hipStream_t st) {
    using L = fse::Launch<R>;
    const fse::GridGeom g = geom(p);
    const void *Dx = nullptr, *Dy = nullptr;
    if (p->Omega != 0.0) {
        HIPCHK(deriv_axis<R>(p, 0, v, b.Dx, st));
        HIPCHK(deriv_axis<R>(p, 1, v, b.Dy, st));
        Dx = b.Dx;
        Dy = b.Dy;
    }
    // W v - Omega Lz v folded into the forward pass of axis 0, P_Delta's
    // inner passes, and v + (.) folded into the inverse pass of axis 0
    const int N0 = p->N[0], NL = p->last();
    HIPCHK(L::gs_cols(1, N0, v, Dx, Dy, b.W, nullptr, b.A, p->C0, g, p->Omega, p->tw[N0], st));
    if (p->d == 3) HIPCHK(L::strided(p->N[1], false, 0, b.A, b.A, N0, p->N[2], p->tw[p->N[1]], nullptr, st));
    HIPCHK(L::line(NL, 1, b.A, (int)p->lines_last(), p->pd, kin_index(p), p->tw[NL], nullptr, st, p->sched[0]));
    if (p->d == 3) HIPCHK(L::strided(p->N[1], true, 0, b.A, b.A, N0, p->N[2], p->tw[p->N[1]], nullptr, st));
    HIPCHK(L::gs_cols(2, N0, v, nullptr, nullptr, nullptr, b.A, out, p->C0, g, 0.0, p->tw[N0], st));
    return FSE_OK;
}

struct Cplx {
    double re, im;
};
inline Cplx cdiv(Cplx a, Cplx b) {
    const double d = b.re * b.re + b.im * b.im;
    return Cplx{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
inline Cplx cmul(Cplx a, Cplx b) { return Cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// Inner products conj(a_k).b_k of npair pairs, read back to the host.
template <typename R> fse_status gs_dots(fse_plan p, int npair, const void* const* a, const void* const* b, Cplx* out,
                                         hipStream_t st) {
    using L = fse::Launch<R>;
    HIPCHK(L::gs_dots(a[0], b[0], npair > 1 ? a[1] : nullptr, npair > 1 ? b[1] : nullptr, npair > 2 ? a[2] : nullptr,
                      npair > 2 ? b[2] : nullptr, npair, p->n, p->partials, kRedBlocks, st));
    HIPCHK(fse::launch_gs_slots(p->partials, kRedBlocks, 2 * npair, 0, p->gs_out, st));
    double h[6];
    HIPCHK(hipMemcpyAsync(h, p->gs_out, sizeof(double) * 2 * npair, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < npair; ++k) out[k] = Cplx{h[2 * k], h[2 * k + 1]};
    return FSE_OK;
}

template <typename R> fse_status gs_step_impl(fse_plan p, void* psi, double dt, double tol, int maxit,
                                              fse_gs_stats* stats, hipStream_t st) {
    using L = fse::Launch<R>;
    GsBuf b;
    fse_status s = ensure_gs(p, &b);
    if (s != FSE_OK) return s;
    const fse::GridGeom g = geom(p);
    const size_t bytes = (size_t)p->n * p->csize;
    const double c0 = 1.0 / dt;
    // frozen W^n = V + beta rho^n + lambda Phi^n
    if (p->nl) {
        if ((s = potential_impl<R>(p, psi, 1, b.Phi, kFrame, 0.0, st)) != FSE_OK) return s;
    }
    hipError_t ee;
    const void* Ux = extra_potential<R>(p, kFrame, st, &ee);
    HIPCHK(ee);
    HIPCHK(L::gs_frozen(psi, p->nl ? b.Phi : nullptr, Ux, b.W, p->n, g, p->beta, p->lambda, p->gamma[0], p->gamma[1],
                        (p->d == 3) ? p->gamma[2] : 0.0, st));
    if ((s = pd_table<R>(p, c0, st)) != FSE_OK) return s;
    // right-hand side P_Delta psi/dt, held in sv until r is formed
    HIPCHK(L::gs_axpy(psi, psi, b.sv, p->n, c0 - 1.0, 0.0, st));  // sv = psi/dt
    if ((s = pd_apply<R>(p, b.sv, st)) != FSE_OK) return s;
    // x0 = psi, r = rhs - M x0, r0 = p = r
    HIPCHK(hipMemcpyAsync(b.x, psi, bytes, hipMemcpyDeviceToDevice, st));
    if ((s = gs_apply_M<R>(p, b, b.x, b.v, st)) != FSE_OK) return s;
    HIPCHK(L::gs_axpy(b.sv, b.v, b.r, p->n, -1.0, 0.0, st));
    HIPCHK(hipMemcpyAsync(b.r0, b.r, bytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(b.pv, b.r, bytes, hipMemcpyDeviceToDevice, st));
    Cplx d3[3];
    {
        const void* a[3] = {b.r0, b.r, b.sv};
        const void* c[3] = {b.r, b.r, b.sv};
        if ((s = gs_dots<R>(p, 3, a, c, d3, st)) != FSE_OK) return s;
    }
    Cplx rho = d3[0];
    const double bnorm = std::sqrt(d3[2].re);
    if (!(bnorm > 0.0)) return fail(FSE_ERR_NUMERIC, "psi is zero");
    double res = std::sqrt(d3[1].re) / bnorm;
    int it = 0;
    bool conv = res <= tol;
    while (!conv && it < maxit) {
        ++it;
        if ((s = gs_apply_M<R>(p, b, b.pv, b.v, st)) != FSE_OK) return s;
        Cplx r0v;
        {
            const void* a[1] = {b.r0};
            const void* c[1] = {b.v};
            if ((s = gs_dots<R>(p, 1, a, c, &r0v, st)) != FSE_OK) return s;
        }
        if (r0v.re == 0.0 && r0v.im == 0.0) return fail(FSE_ERR_NUMERIC, "BiCGStab breakdown: (r0, v) = 0");
        const Cplx alpha = cdiv(rho, r0v);
        HIPCHK(L::gs_axpy(b.r, b.v, b.sv, p->n, -alpha.re, -alpha.im, st));  // s = r - alpha v
        Cplx ss;
        {
            const void* a[1] = {b.sv};
            if ((s = gs_dots<R>(p, 1, a, a, &ss, st)) != FSE_OK) return s;
        }
        if (std::sqrt(ss.re) / bnorm <= tol) {
            HIPCHK(L::gs_axpy(b.x, b.pv, b.x, p->n, alpha.re, alpha.im, st));  // x += alpha p
            res = std::sqrt(ss.re) / bnorm;
            conv = true;
            break;
        }
        if ((s = gs_apply_M<R>(p, b, b.sv, b.t, st)) != FSE_OK) return s;
        Cplx ts_tt[2];
        {
            const void* a[2] = {b.t, b.t};
            const void* c[2] = {b.sv, b.t};
            if ((s = gs_dots<R>(p, 2, a, c, ts_tt, st)) != FSE_OK) return s;
        }
        if (ts_tt[1].re == 0.0) return fail(FSE_ERR_NUMERIC, "BiCGStab breakdown: (t, t) = 0");
        const Cplx omega{ts_tt[0].re / ts_tt[1].re, ts_tt[0].im / ts_tt[1].re};
        HIPCHK(L::gs_update_xr(b.x, b.r, b.pv, b.sv, b.t, p->n, alpha.re, alpha.im, omega.re, omega.im, st));
        Cplx rr[2];
        {
            const void* a[2] = {b.r0, b.r};
            const void* c[2] = {b.r, b.r};
            if ((s = gs_dots<R>(p, 2, a, c, rr, st)) != FSE_OK) return s;
        }
        res = std::sqrt(rr[1].re) / bnorm;
        if (res <= tol) {
            conv = true;
            break;
        }
        if ((omega.re == 0.0 && omega.im == 0.0) || (rho.re == 0.0 && rho.im == 0.0))
            return fail(FSE_ERR_NUMERIC, "BiCGStab breakdown: omega = 0 or rho = 0");
        const Cplx beta = cmul(cdiv(rr[0], rho), cdiv(alpha, omega));
        HIPCHK(L::gs_update_p(b.pv, b.r, b.v, p->n, beta.re, beta.im, omega.re, omega.im, st));
        rho = rr[0];
    }
    // psi <- x / ||x||, ||.||^2 = h^d sum |.|^2
    Cplx xx;
    {
        const void* a[1] = {b.x};
        if ((s = gs_dots<R>(p, 1, a, a, &xx, st)) != FSE_OK) return s;
    }
    double vol = 1.0;
    for (int j = 0; j < p->d; ++j) vol *= p->h[j];
    const double nrm2 = vol * xx.re;
    if (!(nrm2 > 0.0) || !std::isfinite(nrm2)) return fail(FSE_ERR_NUMERIC, "solution has zero or non-finite norm");
    HIPCHK(L::gs_finish(b.x, psi, p->n, 1.0 / std::sqrt(nrm2), p->partials, kRedBlocks, st));
    HIPCHK(fse::launch_gs_slots(p->partials, kRedBlocks, 1, 1, p->gs_out, st));
    double diff = 0.0;
    HIPCHK(hipMemcpyAsync(&diff, p->gs_out, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (stats) {
        stats->iterations = it;
        stats->converged = conv ? 1 : 0;
        stats->residual = res;
        stats->diff_inf = diff;
    }
    return FSE_OK;
}

// The energy E(psi) of eq. energy in the frame of eq. SFSE (the functional the
// gradient flow decreases), reduced on the device in FP64 and read back.
template <typename R> fse_status gs_energy(fse_plan p, const void* psi, double* E, hipStream_t st) {
    fse_status s = reduce_impl<R>(p, psi, 1, p->gs_out, st, kFrame);
    if (s != FSE_OK) return s;
    double e[6];
    HIPCHK(hipMemcpyAsync(e, p->gs_out, sizeof(e), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *E = e[5];
    return FSE_OK;
}

// Ground-state steps until a stopping rule holds after a step: the paper's
// ||phi^n - phi^{n+1}||_inf <= eps_diff dt (Section 3.3), or an energy change
// |E^{n+1} - E^n| <= eps_energy; rules with a tolerance <= 0 are not used.
template <typename R>
fse_status gs_run_impl(fse_plan p, void* psi, double dt, double tol, int maxit, int max_steps, double eps_diff,
                       double eps_energy, double* trace, fse_gs_run_stats* rs, hipStream_t st) {
    GsBuf b;
    fse_status s = ensure_gs(p, &b);
    if (s != FSE_OK) return s;
    const bool want_e = eps_energy > 0.0 || trace != nullptr;
    double E = NAN, dE = NAN;
    if (want_e && (s = gs_energy<R>(p, psi, &E, st)) != FSE_OK) return s;
    if (trace) trace[0] = E;
    fse_gs_stats s1{};
    int n = 0, rule = 0;
    long its = 0;
    while (n < max_steps) {
        if ((s = gs_step_impl<R>(p, psi, dt, tol, maxit, &s1, st)) != FSE_OK) return s;
        ++n;
        its += s1.iterations;
        if (want_e) {
            const double Eprev = E;
            if ((s = gs_energy<R>(p, psi, &E, st)) != FSE_OK) return s;
            dE = std::fabs(E - Eprev);
            if (trace) trace[n] = E;
        }
        if (eps_diff > 0.0 && s1.diff_inf <= eps_diff * dt) {
            rule = 1;
            break;
        }
        if (eps_energy > 0.0 && dE <= eps_energy) {
            rule = 2;
            break;
        }
    }
    if (rs) {
        rs->steps = n;
        rs->converged = rule != 0;
        rs->rule = rule;
        rs->krylov_iterations = (int)std::min<long>(its, 0x7fffffffL);
        rs->diff_inf = s1.diff_inf;
        rs->energy = E;
        rs->energy_change = dE;
        rs->residual = s1.residual;
    }
    return FSE_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free mass reduction (fse_mass_noalloc): the per-block partial
// sums live in a fixed device array instead of the plan's buffer.  Host code
// never passes the array's name to a kernel (in host code it names a host-side
// stand-in); its device address is taken once per device with
// hipGetSymbolAddress and kept.  Every call on a device shares that device's
// array, so calls that overlap on one device race.
// ---------------------------------------------------------------------------
constexpr int kNoallocSlots = 4;  // k_red_local writes four slots per block
static __device__ __align__(256) double scratch[kNoallocSlots * kRedBlocks];
constexpr size_t kScratchBytes = sizeof(double) * kNoallocSlots * kRedBlocks;

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_dev;  // device ordinal -> address of that device's scratch

fse_status scratch_address(double** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_dev.find(dev);
    if (it == g_scratch_dev.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(FSE_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        it = g_scratch_dev.emplace(dev, static_cast<double*>(ptr)).first;
    }
    *out = it->second;
    return FSE_OK;
}

template <typename R> fse_status mass_noalloc_impl(fse_plan p, const void* psi, double* out, hipStream_t st) {
    // the partials this reduction writes: kNoallocSlots slots of kRedBlocks blocks, whatever the grid size
    const size_t need = sizeof(double) * kNoallocSlots * kRedBlocks;
    if (need > kScratchBytes)
        return fail(FSE_ERR_ARG, "the reduction needs %zu bytes of scratch, more than the %zu available", need,
                    kScratchBytes);
    double* sp = nullptr;
    if (fse_status s = scratch_address(&sp); s != FSE_OK) return s;
    const double vol = p->h[0] * p->h[1] * ((p->d == 3) ? p->h[2] : 1.0);
    HIPCHK(fse::Launch<R>::red_local(psi, nullptr, nullptr, p->n, geom(p), 0, 0, 0, 0, nullptr, 0, 0, sp, 0, kRedBlocks,
                                     st));
    HIPCHK(fse::launch_red_final(sp, kRedBlocks, 1, 0, vol, (double)p->n, p->beta, p->lambda, p->Omega, out, st));
    return FSE_OK;
}

void destroy(fse_plan p) {
    if (!p) return;
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    if (p->guard_ev) (void)hipEventDestroy(p->guard_ev);
    if (p->guard_host) (void)hipHostFree(p->guard_host);
    for (void* a : p->allocs) (void)hipFree(a);
    delete p;
}

}  // namespace

static fse_status create_plan(fse_plan* out, int d, const int* N, const double* L, double s, double Omega,
                              const double* gamma, double beta, double lambda, const fse_kernel* kernel, int precision,
                              double m, void* stream, fse_plan donor) {
    if (!out) return fail(FSE_ERR_ARG, "out must not be NULL");
    *out = nullptr;
    fse_status st = check_args(d, N, L, s, Omega, gamma, beta, lambda, kernel, precision);
    if (st != FSE_OK) return st;
    if (!(m >= 0.0) || !std::isfinite(m)) return fail(FSE_ERR_ARG, "m must be finite and >= 0");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(FSE_ERR_HIP, "no HIP device available");
    fse_plan p = new fse_plan_s();
    p->d = d;
    p->n = 1;
    for (int j = 0; j < d; ++j) {
        p->N[j] = N[j];
        p->L[j] = L[j];
        p->h[j] = 2.0 * L[j] / N[j];
        p->gamma[j] = gamma[j];
        p->n *= N[j];
    }
    p->s = s;
    p->Omega = Omega;
    p->beta = beta;
    p->lambda = lambda;
    p->m = m;
    p->prec = precision;
    p->csize = (precision == FSE_C128) ? 16 : 8;
    p->rsize = p->csize / 2;
    if (kernel) p->kernel = *kernel;
    else p->kernel.kind = FSE_K_NONE;
    p->nl = (p->kernel.kind != FSE_K_NONE) && (lambda != 0.0);
    p->qf = p->nl && dipole_needs_form(&p->kernel, Omega);
    p->C0 = (int)(p->n / N[0]);
    // default schedule: plain radix schedules; the mirrored kinetic visit
    // order in 3D FP64 (measured faster there, slower for the complex64 table)
    p->sched[2] = (d == 3 && precision == FSE_C128) ? 1 : 0;
    for (double& t : p->tune_ms) t = -1.0;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    auto bail = [&](fse_status e) {
        destroy(p);
        return e;
    };
    // twiddles: N_j for every axis, 2 N0 (real-to-complex), 2 N_j for the padded axes
    for (int j = 0; j < d; ++j) {
        if ((st = upload_twiddles(p, N[j])) != FSE_OK) return bail(st);
    }
    if ((st = upload_twiddles(p, 2 * N[0])) != FSE_OK) return bail(st);
    if (p->nl) {
        for (int j = 1; j < d; ++j)
            if ((st = upload_twiddles(p, 2 * N[j])) != FSE_OK) return bail(st);
        for (int j = 0; j < d; ++j)
            if ((st = upload_twiddles(p, N[j])) != FSE_OK) return bail(st);
        if (donor && donor->khat) {
            // same grid and kernel: share the donor's multiplier (not owned here)
            p->khat_host = donor->khat_host;
            p->khat = donor->khat;
        } else if (p->qf) {
            // the Coulomb part of the dipole; the quadratic form is applied per convolution
            const double c = 1.0 / ((d == 3 ? 4.0 : 2.0) * kPi);
            p->khat_host = fse::gausum_symbol(d, N, L, FSE_K_COULOMB, 1.0, c, p->kernel.delta, p->kernel.ht,
                                              p->kernel.n);
        } else {
            p->khat_host = fse::gausum_symbol(d, N, L, p->kernel.kind, p->kernel.mu, p->kernel.prefactor,
                                              p->kernel.delta, p->kernel.ht, p->kernel.n);
        }
        double scale = 1.0;
        for (int j = 0; j < d; ++j) scale /= (2.0 * N[j]);
        p->khat_scale = scale;
        const size_t nk = p->khat_host.size();
        if (p->khat) {
            // shared multiplier: nothing to upload
        } else if ((st = dev_alloc(p, &p->khat, nk * p->rsize)) != FSE_OK) {
            return bail(st);
        } else if (precision == FSE_C128) {
            std::vector<double> v(nk);
            for (size_t i = 0; i < nk; ++i) v[i] = p->khat_host[i] * scale;
            if (hipMemcpy(p->khat, v.data(), nk * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
                return bail(fail(FSE_ERR_HIP, "copy of the GauSum multiplier failed"));
        } else {
            std::vector<float> v(nk);
            for (size_t i = 0; i < nk; ++i) v[i] = (float)(p->khat_host[i] * scale);
            if (hipMemcpy(p->khat, v.data(), nk * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
                return bail(fail(FSE_ERR_HIP, "copy of the GauSum multiplier failed"));
        }
        const size_t x1 = (size_t)(N[0] + 1) * p->C0;
        if ((st = dev_alloc(p, &p->X1, x1 * p->csize)) != FSE_OK) return bail(st);
        if (d == 3) {
            const size_t x2 = (size_t)(N[0] + 1) * 2 * N[1] * N[2];
            if ((st = dev_alloc(p, &p->X2, x2 * p->csize)) != FSE_OK) return bail(st);
        }
    }
    if ((st = dev_alloc(p, (void**)&p->partials, sizeof(double) * kRedBlocks * kRedSlots)) != FSE_OK) return bail(st);
    if ((st = dev_alloc(p, (void**)&p->tdev, sizeof(double))) != FSE_OK) return bail(st);
    if ((st = dev_alloc(p, (void**)&p->renorm, 4 * sizeof(double))) != FSE_OK) return bail(st);
    p->renorm_on = (precision == FSE_C64);
    if (hipStreamSynchronize(hs) != hipSuccess) return bail(fail(FSE_ERR_HIP, "stream synchronisation failed"));
    const double t0 = 0.0;
    if (hipMemcpy(p->tdev, &t0, sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(FSE_ERR_HIP, "copy of the initial time failed"));
    *out = p;
    return FSE_OK;
}


// ---------------------------------------------------------------------------
// Batched 2D sweep.
// ---------------------------------------------------------------------------
struct fse_batch_s {
    int count = 0;
    int prec = FSE_C128;
    size_t csize = 16;
    std::vector<fse_plan> plans;  // one per instance (workspace, kinetic tables, diagnostics)
    std::vector<fse_instance> inst;
    std::vector<size_t> off;      // count + 1 element offsets
    std::vector<double> t_host;
    double* t_dev = nullptr;
    fse::BInst* d_all = nullptr;  // descriptors, grouped
    struct Group {
        int N0 = 0, N1 = 0;
        bool nl = false;
        std::vector<int> idx;
        size_t first = 0;  // index of the group's first descriptor in d_all
        hipStream_t s = nullptr;
        hipEvent_t done = nullptr;
    };
    std::vector<Group> groups;
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr;
    std::map<std::pair<int, void*>, hipGraphExec_t> graphs;
    // FP64 mass renormalisation of a step call (on by default for complex64): per instance
    // {mass at the call's start, factor, mass before the exit pass, -} and kBatchRed partial sums
    bool renorm_on = false;
    double* rn = nullptr;
    double* partials = nullptr;
};

namespace {

void batch_destroy(fse_batch b) {
    if (!b) return;
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& g : b->groups) {
        if (g.s) (void)hipStreamDestroy(g.s);
        if (g.done) (void)hipEventDestroy(g.done);
    }
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->d_all) (void)hipFree(b->d_all);
    if (b->t_dev) (void)hipFree(b->t_dev);
    if (b->rn) (void)hipFree(b->rn);
    if (b->partials) (void)hipFree(b->partials);
    // plans sharing a multiplier do not own it; destroy them after its owner's users
    for (auto it = b->plans.rbegin(); it != b->plans.rend(); ++it) destroy(*it);
    delete b;
}

template <typename R> fse_status batch_record_group(fse_batch b, const fse_batch_s::Group& g, void* psi, int nsteps) {
    using L = fse::Launch<R>;
    const fse_plan rep = b->plans[g.idx[0]];
    const int N0 = g.N0, N1 = g.N1, cnt = (int)g.idx.size();
    const fse::BInst* d = b->d_all + g.first;
    const fse::LineIdx lk{1, N0, 0, 1, N1 / 2 + 1};
    const fse::LineIdx lc{1, 0, 0, 1, N1 + 1};
    void* a0 = rep->tw[N0];
    void* b0 = rep->tw[2 * N0];
    void* a1 = rep->tw[N1];
    void* b1 = g.nl ? rep->tw[2 * N1] : nullptr;
    hipStream_t st = g.s;
    const bool rn = b->renorm_on;
    double* part = b->partials + g.first * kBatchRed;  // (the groups' branches run concurrently: disjoint ranges)
    const long npts = (long)N0 * N1;
    if (rn) HIPCHK(L::batch_mass(0, npts, 1.0, psi, d, cnt, part, kBatchRed, st));
    HIPCHK(L::batch(0, N0, N1, psi, d, cnt, 0, lk, a0, b0, a1, b1, st));
    HIPCHK(L::batch(2, N0, N1, psi, d, cnt, 0, lk, a0, b0, a1, b1, st));
    for (int k = 0; k < nsteps; ++k) {
        if (g.nl) {
            HIPCHK(L::batch(3, N0, N1, psi, d, cnt, 0, lc, a0, b0, a1, b1, st));
            HIPCHK(L::batch(4, N0, N1, psi, d, cnt, 0, lc, a0, b0, a1, b1, st));
            HIPCHK(L::batch(5, N0, N1, psi, d, cnt, k, lc, a0, b0, a1, b1, st));
        } else {
            HIPCHK(L::batch(6, N0, N1, psi, d, cnt, k, lc, a0, b0, a1, b1, st));
        }
        HIPCHK(L::batch(2, N0, N1, psi, d, cnt, (k == nsteps - 1) ? 0 : 1, lk, a0, b0, a1, b1, st));
    }
    // the exit pass applies each instance's factor (which = 1) after the mass before it is taken
    if (rn) HIPCHK(L::batch_mass(1, npts, (double)N0, psi, d, cnt, part, kBatchRed, st));
    HIPCHK(L::batch(1, N0, N1, psi, d, cnt, rn ? 1 : 0, lk, a0, b0, a1, b1, st));
    return FSE_OK;
}

fse_status batch_capture(fse_batch b, void* psi, int nsteps, hipGraphExec_t* exec) {
    HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    fse_status s = FSE_OK;
    auto end_capture = [&]() {
        hipGraph_t gr = nullptr;
        (void)hipStreamEndCapture(b->cap, &gr);
        if (gr) (void)hipGraphDestroy(gr);
    };
    if (hipEventRecord(b->fork, b->cap) != hipSuccess) {
        end_capture();
        return fail(FSE_ERR_HIP, "event record during capture failed");
    }
    for (auto& g : b->groups) {
        if (hipStreamWaitEvent(g.s, b->fork, 0) != hipSuccess) {
            end_capture();
            return fail(FSE_ERR_HIP, "stream fork during capture failed");
        }
        s = (b->prec == FSE_C128) ? batch_record_group<double>(b, g, psi, nsteps)
                                  : batch_record_group<float>(b, g, psi, nsteps);
        if (s != FSE_OK) {
            end_capture();
            return s;
        }
        if (hipEventRecord(g.done, g.s) != hipSuccess || hipStreamWaitEvent(b->cap, g.done, 0) != hipSuccess) {
            end_capture();
            return fail(FSE_ERR_HIP, "stream join during capture failed");
        }
    }
    if (fse::launch_batch_time(b->d_all, b->count, nsteps, b->cap) != hipSuccess) {
        end_capture();
        return fail(FSE_ERR_HIP, "time update launch failed");
    }
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamEndCapture(b->cap, &graph));
    hipError_t e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(FSE_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    return FSE_OK;
}

}  // namespace

extern "C" {

const char* fse_last_error(void) { return g_err.c_str(); }

const char* fse_version(void) { return "fse-mi355x 0.1 (gfx950)"; }

fse_status fse_plan_check(int d, const int* N, const double* L, double s, double Omega, const double* gamma,
                          double beta, double lambda, const fse_kernel* kernel, int precision) {
    g_err.clear();
    return check_args(d, N, L, s, Omega, gamma, beta, lambda, kernel, precision);
}

fse_status fse_gausum_symbol_host(int d, const int* N, const double* L, const fse_kernel* kernel, double* out) {
    g_err.clear();
    if (!kernel || !out) return fail(FSE_ERR_ARG, "kernel and out must not be NULL");
    if (kernel->kind == FSE_K_NONE) return fail(FSE_ERR_ARG, "no kernel");
    const double gam[3] = {0, 0, 0};
    fse_status st = check_args(d, N, L, 1.0, 0.0, gam, 0.0, 1.0, kernel, FSE_C128);
    if (st != FSE_OK) return st;
    if (dipole_needs_form(kernel, 0.0))
        return fail(FSE_ERR_UNSUPPORTED, "a tilted dipole axis has no multiplier even in each frequency");
    std::vector<double> k = fse::gausum_symbol(d, N, L, kernel->kind, kernel->mu, kernel->prefactor, kernel->delta,
                                               kernel->ht, kernel->n);
    std::memcpy(out, k.data(), k.size() * sizeof(double));
    return FSE_OK;
}

fse_status fse_plan_create(fse_plan* out, int d, const int* N, const double* L, double s, double Omega,
                           const double* gamma, double beta, double lambda, const fse_kernel* kernel, int precision,
                           double m, void* stream) {
    g_err.clear();
    return create_plan(out, d, N, L, s, Omega, gamma, beta, lambda, kernel, precision, m, stream, nullptr);
}

fse_status fse_plan_destroy(fse_plan plan) {
    g_err.clear();
    if (!plan) return FSE_OK;
    (void)hipDeviceSynchronize();
    destroy(plan);
    return FSE_OK;
}

// Scratch of the step: X1 and X2 (3D), each rounded up to 256 bytes.
size_t scratch_parts(const fse_plan p, size_t* x1b, size_t* x2b) {
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    *x1b = p->nl ? up((size_t)(p->N[0] + 1) * p->C0 * p->csize) : 0;
    *x2b = (p->nl && p->d == 3) ? up((size_t)(p->N[0] + 1) * 2 * p->N[1] * p->N[2] * p->csize) : 0;
    return *x1b + *x2b;
}

fse_status fse_scratch_size(fse_plan plan, size_t* bytes) {
    g_err.clear();
    if (!plan || !bytes) return fail(FSE_ERR_ARG, "plan and bytes must not be NULL");
    size_t a, b;
    *bytes = scratch_parts(plan, &a, &b);
    return FSE_OK;
}

fse_status fse_set_workspace(fse_plan plan, void* dev_ptr, size_t bytes) {
    g_err.clear();
    if (!plan) return fail(FSE_ERR_ARG, "plan must not be NULL");
    size_t x1b, x2b;
    const size_t need = scratch_parts(plan, &x1b, &x2b);
    if (need == 0) return FSE_OK;  // no nonlocal term: the step has no scratch
    if (dev_ptr && bytes < need)
        return fail(FSE_ERR_ARG, "workspace of %zu bytes is smaller than the %zu the plan needs", bytes, need);
    if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) % 256) != 0)
        return fail(FSE_ERR_ARG, "workspace must be 256-byte aligned");
    // release the current scratch (the plan's own memory, or forget the caller's)
    if (!plan->ext_ws) {
        dev_free(plan, plan->X1, x1b ? (size_t)(plan->N[0] + 1) * plan->C0 * plan->csize : 0);
        if (plan->X2) dev_free(plan, plan->X2, (size_t)(plan->N[0] + 1) * 2 * plan->N[1] * plan->N[2] * plan->csize);
    }
    plan->X1 = plan->X2 = nullptr;
    plan->ext_ws = false;
    if (dev_ptr) {
        plan->X1 = dev_ptr;
        if (x2b) plan->X2 = static_cast<char*>(dev_ptr) + x1b;
        plan->ext_ws = true;
        return FSE_OK;
    }
    fse_status st = dev_alloc(plan, &plan->X1, (size_t)(plan->N[0] + 1) * plan->C0 * plan->csize);
    if (st == FSE_OK && plan->d == 3)
        st = dev_alloc(plan, &plan->X2, (size_t)(plan->N[0] + 1) * 2 * plan->N[1] * plan->N[2] * plan->csize);
    return st;
}

fse_status fse_workspace_size(fse_plan plan, size_t* bytes) {
    if (!plan || !bytes) return fail(FSE_ERR_ARG, "plan and bytes must not be NULL");
    *bytes = plan->bytes;
    return FSE_OK;
}

fse_status fse_set_time(fse_plan plan, double t) {
    g_err.clear();
    if (!plan) return fail(FSE_ERR_ARG, "plan must not be NULL");
    if (!std::isfinite(t)) return fail(FSE_ERR_ARG, "t must be finite");
    return write_time(plan, t);
}

fse_status fse_get_time(fse_plan plan, double* t) {
    g_err.clear();
    if (!plan || !t) return fail(FSE_ERR_ARG, "plan and t must not be NULL");
    return read_time(plan, t);
}

fse_status fse_set_mass_renorm(fse_plan plan, int enable) {
    g_err.clear();
    if (!plan) return fail(FSE_ERR_ARG, "plan must not be NULL");
    plan->renorm_on = enable != 0;
    return FSE_OK;
}

fse_status fse_get_mass_renorm(fse_plan plan, int* enabled, double* factor_mass) {
    g_err.clear();
    if (!plan || !enabled) return fail(FSE_ERR_ARG, "plan and enabled must not be NULL");
    *enabled = plan->renorm_on ? 1 : 0;
    if (factor_mass) {
        double r[3];
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(r, plan->renorm, sizeof(r), hipMemcpyDeviceToHost));
        factor_mass[0] = r[1];
        factor_mass[1] = r[2];
        factor_mass[2] = r[0];
    }
    return FSE_OK;
}

fse_status fse_set_guard(fse_plan plan, double tol) {
    g_err.clear();
    if (!plan) return fail(FSE_ERR_ARG, "plan must not be NULL");
    if (!std::isfinite(tol)) return fail(FSE_ERR_ARG, "tol must be finite");
    if (tol > 0.0) {  // each resource on its own, so that a call after a failed one completes the set
        if (!plan->guard_dev) {
            fse_status s = dev_alloc(plan, reinterpret_cast<void**>(&plan->guard_dev), 3 * sizeof(double));
            if (s != FSE_OK) return s;
        }
        if (!plan->guard_host &&
            hipHostMalloc(reinterpret_cast<void**>(&plan->guard_host), 3 * sizeof(double), hipHostMallocDefault) !=
                hipSuccess) {
            plan->guard_host = nullptr;
            return fail(FSE_ERR_NOMEM, "hipHostMalloc for the guard");
        }
        if (!plan->guard_ev && hipEventCreateWithFlags(&plan->guard_ev, hipEventDisableTiming) != hipSuccess) {
            plan->guard_ev = nullptr;
            return fail(FSE_ERR_HIP, "hipEventCreate for the guard");
        }
    }
    if (plan->guard_dev && plan->guard_host) {
        // no check may still be writing the buffers that are reset here
        if (hipDeviceSynchronize() != hipSuccess) return fail(FSE_ERR_HIP, "hipDeviceSynchronize");
        const double init[3] = {NAN, NAN, 0.0};
        if (hipMemcpy(plan->guard_dev, init, sizeof(init), hipMemcpyHostToDevice) != hipSuccess)
            return fail(FSE_ERR_HIP, "hipMemcpy");
        std::memcpy(plan->guard_host, init, sizeof(init));
    }
    plan->guard_tol = tol > 0.0 ? tol : 0.0;
    plan->guard_pending = plan->guard_tripped = false;
    return FSE_OK;
}

fse_status fse_guard_status(fse_plan plan, int* tripped, double* masses) {
    g_err.clear();
    if (!plan || !tripped) return fail(FSE_ERR_ARG, "plan and tripped must not be NULL");
    if (plan->guard_pending) {
        if (hipEventSynchronize(plan->guard_ev) != hipSuccess) return fail(FSE_ERR_HIP, "hipEventSynchronize");
        plan->guard_pending = false;
        if (plan->guard_host[2] != 0.0) plan->guard_tripped = true;
    }
    *tripped = plan->guard_tripped ? 1 : 0;
    if (masses) {
        masses[0] = plan->guard_host ? plan->guard_host[0] : NAN;
        masses[1] = plan->guard_host ? plan->guard_host[1] : NAN;
    }
    return FSE_OK;
}

fse_status fse_step(fse_plan plan, void* psi, int nsteps, double dt, void* stream) {
    g_err.clear();
    if (!plan || !psi) return fail(FSE_ERR_ARG, "plan and psi must not be NULL");
    if (nsteps < 0) return fail(FSE_ERR_ARG, "nsteps must be >= 0");
    if (!std::isfinite(dt) || dt == 0.0) return fail(FSE_ERR_ARG, "dt must be finite and non-zero");
    if (fse_status s = guard_poll(plan); s != FSE_OK) return s;
    if (nsteps == 0) return FSE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    fse_status s = plan->prec == FSE_C128 ? step_impl<double>(plan, psi, nsteps, dt, 2, st)
                                          : step_impl<float>(plan, psi, nsteps, dt, 2, st);
    return s == FSE_OK ? guard_check(plan, psi, st) : s;
}

fse_status fse_step4(fse_plan plan, void* psi, int nsteps, double dt, void* stream) {
    g_err.clear();
    if (!plan || !psi) return fail(FSE_ERR_ARG, "plan and psi must not be NULL");
    if (nsteps < 0) return fail(FSE_ERR_ARG, "nsteps must be >= 0");
    if (!std::isfinite(dt) || dt == 0.0) return fail(FSE_ERR_ARG, "dt must be finite and non-zero");
    if (fse_status s = guard_poll(plan); s != FSE_OK) return s;
    if (nsteps == 0) return FSE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    fse_status s = plan->prec == FSE_C128 ? step_impl<double>(plan, psi, nsteps, dt, 4, st)
                                          : step_impl<float>(plan, psi, nsteps, dt, 4, st);
    return s == FSE_OK ? guard_check(plan, psi, st) : s;
}

fse_status fse_apply_H(fse_plan plan, const void* psi, void* Hpsi, const void* rho_frozen, void* stream) {
    g_err.clear();
    if (!plan || !psi || !Hpsi) return fail(FSE_ERR_ARG, "plan, psi and Hpsi must not be NULL");
    if (psi == Hpsi) return fail(FSE_ERR_ARG, "psi and Hpsi must not alias");
    if (plan->U && plan->Omega != 0.0)
        return fail(FSE_ERR_UNSUPPORTED, "a grid potential set by fse_set_potential needs Omega = 0 in H psi");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? apply_H_impl<double>(plan, psi, Hpsi, rho_frozen, st)
                                  : apply_H_impl<float>(plan, psi, Hpsi, rho_frozen, st);
}

fse_status fse_gs_step(fse_plan plan, void* psi, double dt, double tol, int maxit, fse_gs_stats* stats,
                       void* stream) {
    g_err.clear();
    if (!plan || !psi) return fail(FSE_ERR_ARG, "plan and psi must not be NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(FSE_ERR_ARG, "dt must be finite and > 0");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FSE_ERR_ARG, "tol must be finite and > 0");
    if (maxit < 1) return fail(FSE_ERR_ARG, "maxit must be >= 1");
    if (plan->U && plan->Omega != 0.0)
        return fail(FSE_ERR_UNSUPPORTED,
                    "a grid potential set by fse_set_potential needs Omega = 0 in the ground-state step");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? gs_step_impl<double>(plan, psi, dt, tol, maxit, stats, st)
                                  : gs_step_impl<float>(plan, psi, dt, tol, maxit, stats, st);
}

fse_status fse_gs_run(fse_plan plan, void* psi, double dt, double tol, int maxit, int max_steps, double eps_diff,
                      double eps_energy, double* energy_trace, fse_gs_run_stats* stats, void* stream) {
    g_err.clear();
    if (!plan || !psi) return fail(FSE_ERR_ARG, "plan and psi must not be NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(FSE_ERR_ARG, "dt must be finite and > 0");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FSE_ERR_ARG, "tol must be finite and > 0");
    if (maxit < 1 || max_steps < 1) return fail(FSE_ERR_ARG, "maxit and max_steps must be >= 1");
    if (!std::isfinite(eps_diff) || !std::isfinite(eps_energy))
        return fail(FSE_ERR_ARG, "eps_diff and eps_energy must be finite");
    if (plan->U && plan->Omega != 0.0)
        return fail(FSE_ERR_UNSUPPORTED,
                    "a grid potential set by fse_set_potential needs Omega = 0 in the ground-state step");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128
               ? gs_run_impl<double>(plan, psi, dt, tol, maxit, max_steps, eps_diff, eps_energy, energy_trace, stats, st)
               : gs_run_impl<float>(plan, psi, dt, tol, maxit, max_steps, eps_diff, eps_energy, energy_trace, stats, st);
}

fse_status fse_nonlocal_potential(fse_plan plan, const void* psi, void* Phi, void* stream) {
    g_err.clear();
    if (!plan || !psi || !Phi) return fail(FSE_ERR_ARG, "plan, psi and Phi must not be NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? potential_impl<double>(plan, psi, 1, Phi, at_plan(), 0.0, st)
                                  : potential_impl<float>(plan, psi, 1, Phi, at_plan(), 0.0, st);
}

fse_status fse_mass(fse_plan plan, const void* psi, double* out_dev, void* stream) {
    g_err.clear();
    if (!plan || !psi || !out_dev) return fail(FSE_ERR_ARG, "plan, psi and out_dev must not be NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? reduce_impl<double>(plan, psi, 0, out_dev, st)
                                  : reduce_impl<float>(plan, psi, 0, out_dev, st);
}

fse_status fse_mass_noalloc(fse_plan plan, const void* psi, double* out_dev, void* stream) {
    g_err.clear();
    if (!plan || !psi || !out_dev) return fail(FSE_ERR_ARG, "plan, psi and out_dev must not be NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? mass_noalloc_impl<double>(plan, psi, out_dev, st)
                                  : mass_noalloc_impl<float>(plan, psi, out_dev, st);
}

fse_status fse_energy(fse_plan plan, const void* psi, double* out_dev, void* stream) {
    g_err.clear();
    if (!plan || !psi || !out_dev) return fail(FSE_ERR_ARG, "plan, psi and out_dev must not be NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? reduce_impl<double>(plan, psi, 1, out_dev, st)
                                  : reduce_impl<float>(plan, psi, 1, out_dev, st);
}

fse_status fse_plan_tune(fse_plan plan, const char* cache_path, void* stream) {
    g_err.clear();
    if (!plan) return fail(FSE_ERR_ARG, "plan must not be NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const std::string key = tune_key(plan);
    if (key.empty()) return fail(FSE_ERR_HIP, "no current device");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end() && cache_path) {
        FILE* f = std::fopen(cache_path, "r");
        if (f) {
            char line[1024];
            while (std::fgets(line, sizeof(line), f)) {
                char* tab = std::strrchr(line, '\t');
                if (!tab) continue;
                *tab = '\0';
                std::array<int, kNSched> v{};
                int used = 0;
                if (key == line &&
                    std::sscanf(tab + 1, "%d %d %d %d %d%n", &v[0], &v[1], &v[2], &v[3], &v[4], &used) == 5 &&
                    std::all_of(v.begin(), v.end(), [](int x) { return x == 0 || x == 1; }))
                    g_tune_cache[key] = v;
            }
            std::fclose(f);
        }
        it = g_tune_cache.find(key);
    }
    if (it != g_tune_cache.end()) {
        for (int k = 0; k < kNSched; ++k) plan->sched[k] = it->second[k];
        for (double& t : plan->tune_ms) t = -1.0;
        return FSE_OK;
    }
    fse_status s = plan->prec == FSE_C128 ? tune_measure<double>(plan, st) : tune_measure<float>(plan, st);
    if (s != FSE_OK) return s;
    g_tune_cache[key] = {plan->sched[0], plan->sched[1], plan->sched[2], plan->sched[3], plan->sched[4]};
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(FSE_ERR_ARG, "cannot append to the tuning cache %s", cache_path);
        std::fprintf(f, "%s\t%d %d %d %d %d\n", key.c_str(), plan->sched[0], plan->sched[1], plan->sched[2],
                     plan->sched[3], plan->sched[4]);
        std::fclose(f);
    }
    return FSE_OK;
}

fse_status fse_plan_get_schedule(fse_plan plan, int* sched, double* tuned_ms) {
    g_err.clear();
    if (!plan || !sched) return fail(FSE_ERR_ARG, "plan and sched must not be NULL");
    for (int k = 0; k < kNSched; ++k) sched[k] = plan->sched[k];
    if (tuned_ms)
        for (int k = 0; k < (1 << kNSched); ++k) tuned_ms[k] = plan->tune_ms[k];
    return FSE_OK;
}

fse_status fse_plan_set_schedule(fse_plan plan, const int* sched) {
    g_err.clear();
    if (!plan || !sched) return fail(FSE_ERR_ARG, "plan and sched must not be NULL");
    for (int k = 0; k < kNSched; ++k)
        if (sched[k] != 0 && sched[k] != 1) return fail(FSE_ERR_ARG, "schedule entries are 0 or 1");
    if (sched[0] == 1 && !kin_has_alt(plan))
        return fail(FSE_ERR_UNSUPPORTED, "line length %d has no alternative radix schedule", plan->last());
    if (sched[1] == 1 && !conv_has_alt(plan))
        return fail(FSE_ERR_UNSUPPORTED, "the convolution of this plan has no alternative radix schedule");
    if (sched[2] == 1 && plan->d != 3) return fail(FSE_ERR_UNSUPPORTED, "the mirrored visit order is 3D only");
    if (sched[3] == 1 && !cols_have_alt(plan))
        return fail(FSE_ERR_UNSUPPORTED, "the column transforms of this plan have no alternative radix plan");
    if (sched[4] == 1 && !fused_has_alt(plan))
        return fail(FSE_ERR_UNSUPPORTED, "the fused phase pass of this plan has no second radix plan");
    for (int k = 0; k < kNSched; ++k) plan->sched[k] = sched[k];
    return FSE_OK;
}

fse_status fse_set_lattice(fse_plan plan, const double* v, const double* k) {
    g_err.clear();
    if (!plan) return fail(FSE_ERR_ARG, "plan must not be NULL");
    if (!v) {
        plan->lat = false;
        return FSE_OK;
    }
    if (!k) return fail(FSE_ERR_ARG, "k must not be NULL when v is given");
    for (int j = 0; j < plan->d; ++j)
        if (!std::isfinite(v[j]) || !std::isfinite(k[j])) return fail(FSE_ERR_ARG, "lattice v and k must be finite");
    if (!plan->lat_buf) {
        fse_status s = dev_alloc(plan, &plan->lat_buf, (size_t)plan->n * plan->rsize);
        if (s != FSE_OK) return s;
    }
    for (int j = 0; j < 3; ++j) {
        plan->lat_v[j] = (j < plan->d) ? v[j] : 0.0;
        plan->lat_k[j] = (j < plan->d) ? k[j] : 0.0;
    }
    plan->lat = true;
    return FSE_OK;
}

fse_status fse_set_potential(fse_plan plan, const void* U) {
    g_err.clear();
    if (!plan) return fail(FSE_ERR_ARG, "plan must not be NULL");
    plan->U = U;
    return FSE_OK;
}

fse_status fse_step_adjoint(fse_plan plan, const void* psi0, int nsteps, double dt, void* grad, void* grad_U,
                            void* stream) {
    g_err.clear();
    if (!plan || !psi0 || !grad) return fail(FSE_ERR_ARG, "plan, psi0 and grad must not be NULL");
    if (psi0 == grad) return fail(FSE_ERR_ARG, "psi0 and grad must not alias");
    if (nsteps < 0) return fail(FSE_ERR_ARG, "nsteps must be >= 0");
    if (!std::isfinite(dt) || dt == 0.0) return fail(FSE_ERR_ARG, "dt must be finite and non-zero");
    if (nsteps == 0) return FSE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? adjoint_impl<double>(plan, psi0, nsteps, dt, grad, grad_U, st)
                                  : adjoint_impl<float>(plan, psi0, nsteps, dt, grad, grad_U, st);
}

fse_status fse_apply_Lz(fse_plan plan, const void* psi, void* out, void* stream) {
    g_err.clear();
    if (!plan || !psi || !out) return fail(FSE_ERR_ARG, "plan, psi and out must not be NULL");
    if (psi == out) return fail(FSE_ERR_ARG, "psi and out must not alias");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? apply_Lz_impl<double>(plan, psi, out, st)
                                  : apply_Lz_impl<float>(plan, psi, out, st);
}

fse_status fse_angular_momentum_grad(fse_plan plan, const void* psi, const double* g_dev, void* out, void* stream) {
    g_err.clear();
    if (!plan || !psi || !out) return fail(FSE_ERR_ARG, "plan, psi and out must not be NULL");
    if (psi == out) return fail(FSE_ERR_ARG, "psi and out must not alias");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double vol = plan->h[0] * plan->h[1] * ((plan->d == 3) ? plan->h[2] : 1.0);
    return plan->prec == FSE_C128 ? apply_Lz_impl<double>(plan, psi, out, st, 2.0 * vol, g_dev)
                                  : apply_Lz_impl<float>(plan, psi, out, st, 2.0 * vol, g_dev);
}

fse_status fse_moments(fse_plan plan, const void* psi, double* out_dev, void* stream) {
    g_err.clear();
    if (!plan || !psi || !out_dev) return fail(FSE_ERR_ARG, "plan, psi and out_dev must not be NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? moments_impl<double>(plan, psi, out_dev, st)
                                  : moments_impl<float>(plan, psi, out_dev, st);
}

fse_status fse_angular_momentum(fse_plan plan, const void* psi, double* out_dev, void* stream) {
    g_err.clear();
    if (!plan || !psi || !out_dev) return fail(FSE_ERR_ARG, "plan, psi and out_dev must not be NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return plan->prec == FSE_C128 ? reduce_impl<double>(plan, psi, 2, out_dev, st)
                                  : reduce_impl<float>(plan, psi, 2, out_dev, st);
}


fse_status fse_batch_create(fse_batch* out, int count, const fse_instance* inst, int precision, void* stream) {
    g_err.clear();
    if (!out || !inst || count < 1) return fail(FSE_ERR_ARG, "out, inst must not be NULL and count >= 1");
    *out = nullptr;
    if (precision != FSE_C128 && precision != FSE_C64) return fail(FSE_ERR_ARG, "unknown precision %d", precision);
    for (int i = 0; i < count; ++i) {
        const fse_instance& q = inst[i];
        fse_status st = check_args(2, q.N, q.L, q.s, q.Omega, q.gamma, q.beta, q.lambda, &q.kernel, precision);
        if (st != FSE_OK) {
            const std::string m = g_err;
            return fail(st, "instance %d: %s", i, m.c_str());
        }
        if (!std::isfinite(q.dt) || q.dt == 0.0) return fail(FSE_ERR_ARG, "instance %d: dt must be finite, non-zero", i);
        if (!(q.m >= 0.0) || !std::isfinite(q.m)) return fail(FSE_ERR_ARG, "instance %d: m must be finite, >= 0", i);
        if (q.lambda != 0.0 && dipole_needs_form(&q.kernel, q.Omega))
            return fail(FSE_ERR_UNSUPPORTED, "instance %d: the batch does not take tilted or turning dipole axes", i);
    }
    fse_batch b = new fse_batch_s();
    b->count = count;
    b->prec = precision;
    b->csize = (precision == FSE_C128) ? 16 : 8;
    b->inst.assign(inst, inst + count);
    b->off.assign(count + 1, 0);
    b->t_host.assign(count, 0.0);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    auto bail = [&](fse_status e) {
        const std::string m = g_err;
        batch_destroy(b);
        g_err = m;
        return e;
    };
    for (int i = 0; i < count; ++i) {
        const fse_instance& q = inst[i];
        b->off[i + 1] = b->off[i] + (size_t)q.N[0] * q.N[1];
        fse_plan donor = nullptr;
        for (int j = 0; j < i; ++j) {
            const fse_instance& r = inst[j];
            if (r.N[0] == q.N[0] && r.N[1] == q.N[1] && r.L[0] == q.L[0] && r.L[1] == q.L[1] &&
                r.kernel.kind == q.kernel.kind && r.kernel.mu == q.kernel.mu &&
                r.kernel.prefactor == q.kernel.prefactor && r.kernel.delta == q.kernel.delta &&
                r.kernel.ht == q.kernel.ht && r.kernel.n[0] == q.kernel.n[0] && r.kernel.n[1] == q.kernel.n[1] &&
                r.kernel.n[2] == q.kernel.n[2] && b->plans[j]->khat) {
                donor = b->plans[j];
                break;
            }
        }
        fse_plan p = nullptr;
        fse_status st = create_plan(&p, 2, q.N, q.L, q.s, q.Omega, q.gamma, q.beta, q.lambda, &q.kernel, precision,
                                    q.m, stream, donor);
        if (st != FSE_OK) return bail(st);
        b->plans.push_back(p);
        void* tab = nullptr;
        st = (precision == FSE_C128) ? kin_table<double>(p, 0.5 * q.dt, 0, &tab, hs)
                                     : kin_table<float>(p, 0.5 * q.dt, 0, &tab, hs);
        if (st != FSE_OK) return bail(st);
        st = (precision == FSE_C128) ? kin_table<double>(p, q.dt, 1, &tab, hs) : kin_table<float>(p, q.dt, 1, &tab, hs);
        if (st != FSE_OK) return bail(st);
    }
    // groups of equal size (and presence of the nonlocal term)
    for (int i = 0; i < count; ++i) {
        const fse_plan p = b->plans[i];
        bool placed = false;
        for (auto& g : b->groups)
            if (g.N0 == p->N[0] && g.N1 == p->N[1] && g.nl == p->nl) {
                g.idx.push_back(i);
                placed = true;
                break;
            }
        if (!placed) {
            fse_batch_s::Group g;
            g.N0 = p->N[0];
            g.N1 = p->N[1];
            g.nl = p->nl;
            g.idx.push_back(i);
            b->groups.push_back(g);
        }
    }
    if (hipMalloc((void**)&b->t_dev, sizeof(double) * count) != hipSuccess) return bail(fail(FSE_ERR_NOMEM, "hipMalloc"));
    if (hipMemset(b->t_dev, 0, sizeof(double) * count) != hipSuccess) return bail(fail(FSE_ERR_HIP, "hipMemset"));
    for (int i = 0; i < count; ++i) b->plans[i]->tdev = b->t_dev + i;  // the diagnostics read the instance's time
    if (hipMalloc((void**)&b->rn, sizeof(double) * 4 * count) != hipSuccess ||
        hipMalloc((void**)&b->partials, sizeof(double) * kBatchRed * count) != hipSuccess)
        return bail(fail(FSE_ERR_NOMEM, "hipMalloc"));
    {
        std::vector<double> r0(4 * (size_t)count, 1.0);  // factor 1 until a renormalising call sets it
        if (hipMemcpy(b->rn, r0.data(), sizeof(double) * r0.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(FSE_ERR_HIP, "hipMemcpy"));
    }
    b->renorm_on = (precision == FSE_C64);
    std::vector<fse::BInst> desc;
    for (auto& g : b->groups) {
        g.first = desc.size();
        for (int i : g.idx) {
            const fse_plan p = b->plans[i];
            const fse_instance& q = inst[i];
            fse::BInst d{};
            d.psi_off = (long)b->off[i];
            d.X1 = p->X1;
            d.khat = p->khat;
            d.kin0 = p->kin[0];
            d.kin1 = p->kin[1];
            d.t = b->t_dev + i;
            d.dt = q.dt;
            d.Omega = q.Omega;
            const double gx2 = q.gamma[0] * q.gamma[0], gy2 = q.gamma[1] * q.gamma[1];
            d.ca = q.dt * (gx2 + gy2) / 4.0;
            d.gdiff = (gx2 - gy2) / 4.0;
            d.sf = (q.Omega == 0.0) ? q.dt : std::sin(q.Omega * q.dt) / q.Omega;
            d.bdt = q.beta * q.dt;
            d.ldt = q.lambda * q.dt;
            d.x0 = -q.L[0];
            d.hx = p->h[0];
            d.y0 = -q.L[1];
            d.hy = p->h[1];
            d.rn = b->rn + 4 * i;
            desc.push_back(d);
        }
        if (hipStreamCreateWithFlags(&g.s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess)
            return bail(fail(FSE_ERR_HIP, "stream/event creation failed"));
    }
    if (hipMalloc((void**)&b->d_all, sizeof(fse::BInst) * desc.size()) != hipSuccess)
        return bail(fail(FSE_ERR_NOMEM, "hipMalloc"));
    if (hipMemcpy(b->d_all, desc.data(), sizeof(fse::BInst) * desc.size(), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(FSE_ERR_HIP, "descriptor upload failed"));
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        return bail(fail(FSE_ERR_HIP, "stream/event creation failed"));
    if (hipStreamSynchronize(hs) != hipSuccess) return bail(fail(FSE_ERR_HIP, "stream synchronisation failed"));
    *out = b;
    return FSE_OK;
}

fse_status fse_batch_destroy(fse_batch batch) {
    g_err.clear();
    if (!batch) return FSE_OK;
    (void)hipDeviceSynchronize();
    batch_destroy(batch);
    return FSE_OK;
}

fse_status fse_batch_offsets(fse_batch batch, size_t* offsets) {
    g_err.clear();
    if (!batch || !offsets) return fail(FSE_ERR_ARG, "batch and offsets must not be NULL");
    for (int i = 0; i <= batch->count; ++i) offsets[i] = batch->off[i];
    return FSE_OK;
}

fse_status fse_batch_times(fse_batch batch, double* t) {
    g_err.clear();
    if (!batch || !t) return fail(FSE_ERR_ARG, "batch and t must not be NULL");
    for (int i = 0; i < batch->count; ++i) t[i] = batch->t_host[i];
    return FSE_OK;
}

fse_status fse_batch_set_mass_renorm(fse_batch batch, int enable) {
    g_err.clear();
    if (!batch) return fail(FSE_ERR_ARG, "batch must not be NULL");
    if ((enable != 0) != batch->renorm_on) {
        // the captured graphs carry the setting: record them again
        HIPCHK(hipDeviceSynchronize());
        for (auto& kv : batch->graphs) (void)hipGraphExecDestroy(kv.second);
        batch->graphs.clear();
        batch->renorm_on = enable != 0;
    }
    return FSE_OK;
}

fse_status fse_batch_get_mass_renorm(fse_batch batch, int* enabled, double* factor_mass) {
    g_err.clear();
    if (!batch || !enabled) return fail(FSE_ERR_ARG, "batch and enabled must not be NULL");
    *enabled = batch->renorm_on ? 1 : 0;
    if (factor_mass) {
        std::vector<double> r(4 * (size_t)batch->count);
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(r.data(), batch->rn, sizeof(double) * r.size(), hipMemcpyDeviceToHost));
        for (int i = 0; i < batch->count; ++i) {  // (the order of fse_get_mass_renorm)
            factor_mass[3 * i] = r[4 * i + 1];
            factor_mass[3 * i + 1] = r[4 * i + 2];
            factor_mass[3 * i + 2] = r[4 * i];
        }
    }
    return FSE_OK;
}

fse_status fse_batch_step(fse_batch batch, void* psi_packed, int nsteps, void* stream) {
    g_err.clear();
    if (!batch || !psi_packed) return fail(FSE_ERR_ARG, "batch and psi_packed must not be NULL");
    if (nsteps < 0) return fail(FSE_ERR_ARG, "nsteps must be >= 0");
    if (nsteps == 0) return FSE_OK;
    const auto key = std::make_pair(nsteps, psi_packed);
    auto it = batch->graphs.find(key);
    hipGraphExec_t exec = nullptr;
    if (it == batch->graphs.end()) {
        if (batch->graphs.size() >= 8) {
            HIPCHK(hipDeviceSynchronize());
            for (auto& kv : batch->graphs) (void)hipGraphExecDestroy(kv.second);
            batch->graphs.clear();
        }
        fse_status s = batch_capture(batch, psi_packed, nsteps, &exec);
        if (s != FSE_OK) return s;
        batch->graphs[key] = exec;
    } else {
        exec = it->second;
    }
    HIPCHK(hipGraphLaunch(exec, static_cast<hipStream_t>(stream)));
    for (int i = 0; i < batch->count; ++i) batch->t_host[i] += nsteps * batch->inst[i].dt;
    return FSE_OK;
}

fse_status fse_batch_reduce(fse_batch batch, const void* psi_packed, double* out_dev, void* stream) {
    g_err.clear();
    if (!batch || !psi_packed || !out_dev) return fail(FSE_ERR_ARG, "batch, psi_packed and out_dev must not be NULL");
    const char* base = static_cast<const char*>(psi_packed);
    for (int i = 0; i < batch->count; ++i) {
        fse_plan p = batch->plans[i];  // (its device time is the instance's entry of the batch's array)
        const void* psi = base + batch->off[i] * batch->csize;
        hipStream_t st = static_cast<hipStream_t>(stream);
        fse_status s = (p->prec == FSE_C128) ? reduce_impl<double>(p, psi, 0, out_dev + 7 * i, st)
                                             : reduce_impl<float>(p, psi, 0, out_dev + 7 * i, st);
        if (s != FSE_OK) return s;
        s = (p->prec == FSE_C128) ? reduce_impl<double>(p, psi, 1, out_dev + 7 * i + 1, st)
                                  : reduce_impl<float>(p, psi, 1, out_dev + 7 * i + 1, st);
        if (s != FSE_OK) return s;
    }
    return FSE_OK;
}

fse_status fse_set_profiling(fse_plan plan, int enable) {
    g_err.clear();
    if (!plan) return fail(FSE_ERR_ARG, "plan must not be NULL");
    plan->prof = enable != 0;
    plan->ev_used = 0;
    return FSE_OK;
}

fse_status fse_get_profile(fse_plan plan, double* ms, int* count, int npass) {
    g_err.clear();
    if (!plan || !ms || !count || npass < 0) return fail(FSE_ERR_ARG, "invalid arguments");
    for (size_t i = 0; i + 1 < plan->ev_used; i += 2) {
        HIPCHK(hipEventSynchronize(plan->ev[i + 1]));
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, plan->ev[i], plan->ev[i + 1]));
        const int k = plan->ev_kind[i / 2];
        if (k < npass) {
            ms[k] += t;
            count[k] += 1;
        }
    }
    plan->ev_used = 0;
    return FSE_OK;
}

fse_status fse_device_copy(void* dst, const void* src, size_t bytes, void* stream) {
    g_err.clear();
    if (!dst || !src) return fail(FSE_ERR_ARG, "dst and src must not be NULL");
    if ((bytes % 16) != 0 || ((uintptr_t)dst % 16) != 0 || ((uintptr_t)src % 16) != 0)
        return fail(FSE_ERR_ARG, "bytes and both pointers must be multiples of 16");
    if (bytes == 0) return FSE_OK;
    HIPCHK(fse::launch_copy16(dst, src, (long)(bytes / 16), static_cast<hipStream_t>(stream)));
    return FSE_OK;
}

fse_status fse_device_copy_nt(void* dst, const void* src, size_t bytes, void* stream) {
    g_err.clear();
    if (!dst || !src) return fail(FSE_ERR_ARG, "dst and src must not be NULL");
    if ((bytes % 16) != 0 || ((uintptr_t)dst % 16) != 0 || ((uintptr_t)src % 16) != 0)
        return fail(FSE_ERR_ARG, "bytes and both pointers must be multiples of 16");
    if (bytes == 0) return FSE_OK;
    HIPCHK(fse::launch_copy16(dst, src, (long)(bytes / 16), static_cast<hipStream_t>(stream), true));
    return FSE_OK;
}

fse_status fse_get_symbol(fse_plan plan, double* host_out) {
    g_err.clear();
    if (!plan || !host_out) return fail(FSE_ERR_ARG, "plan and host_out must not be NULL");
    if (!plan->nl) return fail(FSE_ERR_STATE, "the plan has no nonlocal kernel");
    std::memcpy(host_out, plan->khat_host.data(), plan->khat_host.size() * sizeof(double));
    return FSE_OK;
}

}  // extern "C"
