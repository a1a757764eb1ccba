// Complex128 instantiation of the split-step kernels.
#define FSE_REAL double
#include "fse_launch.inc"

namespace fse {

static bool in_list(int M, const int* l, int n) {
    for (int i = 0; i < n; ++i)
        if (l[i] == M) return true;
    return false;
}

bool strided_size_ok(int M) {
    static const int l[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
    return in_list(M, l, sizeof(l) / sizeof(l[0]));
}

bool line_size_ok(int M) { return strided_size_ok(M); }

hipError_t launch_batch_time(const BInst* bi, int count, int nsteps, hipStream_t st) {
    k_b_time<<<(count + 63) / 64, 64, 0, st>>>(bi, count, nsteps);
    return hipGetLastError();
}

hipError_t launch_b_mass_final(const double* partials, int nblk, const BInst* bi, int count, double mscale, int slot,
                               hipStream_t st) {
    k_b_mass_final<<<(unsigned)count, RED_THREADS, 0, st>>>(partials, nblk, bi, mscale, slot);
    return hipGetLastError();
}

hipError_t launch_gs_slots(const double* partials, int nblk, int nslot, int op, double* out, hipStream_t st) {
    k_gs_slots<<<(unsigned)nslot, RED_THREADS, 0, st>>>(partials, nblk, op, out);
    return hipGetLastError();
}

bool line_has_alt(int n) {
    switch (n) {
#define ALT_CASE(NN) \
    case NN:         \
        return AltRadix<NN>::has;
        FSE_N_SIZES(ALT_CASE)
#undef ALT_CASE
        default:
            return false;
    }
}

bool col_has_alt(int n) {
    switch (n) {
#define ALT_CASE(NN) \
    case NN:         \
        return ColPlanOf<NN>::has_alt;
        FSE_N_SIZES(ALT_CASE)
#undef ALT_CASE
        default:
            return false;
    }
}

bool fused_has_alt(int n) {
    switch (n) {
#define ALT_CASE(NN) \
    case NN:         \
        return FusedPlan<double, NN, 0>::has_alt;
        FSE_N_SIZES(ALT_CASE)
#undef ALT_CASE
        default:
            return false;
    }
}

hipError_t launch_copy16(void* dst, const void* src, long n16, hipStream_t st, bool nontemporal) {
    const long g = (n16 + 1023) / 1024;  // 1024 elements per workgroup
    if (g > 0x7fffffffL) return hipErrorInvalidValue;
    if (nontemporal)
        k_copy16<true><<<(unsigned)g, 256, 0, st>>>(static_cast<double2*>(dst), static_cast<const double2*>(src), n16);
    else
        k_copy16<false><<<(unsigned)g, 256, 0, st>>>(static_cast<double2*>(dst), static_cast<const double2*>(src), n16);
    return hipGetLastError();
}

hipError_t launch_red_final(const double* partials, int nblk, int nslot, int kind, double vol, double n,
                            double beta, double lam, double Omega, double* out, hipStream_t st) {
    k_red_final<<<1, RED_THREADS, 0, st>>>(partials, nblk, nslot, kind, vol, n, beta, lam, Omega, out);
    return hipGetLastError();
}

__global__ void k_zero8(unsigned long long* __restrict__ p, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0ull;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    if (bytes % 8 != 0) return hipErrorInvalidValue;
    const long n = (long)(bytes / 8);
    if (n == 0) return hipSuccess;
    const long blocks = std::min<long>((n + 255) / 256, 4096);
    k_zero8<<<(unsigned)blocks, 256, 0, st>>>(static_cast<unsigned long long*>(p), n);
    return hipGetLastError();
}

__global__ void k_guard(double* g, double tol) {
    if (threadIdx.x == 0) {
        const double m = g[1];
        if (isnan(g[0])) g[0] = m;
        const double m0 = g[0];
        if (!isfinite(m) || !isfinite(m0) || fabs(m - m0) > tol * fabs(m0)) g[2] = 1.0;
    }
}

hipError_t launch_guard(double* g, double tol, hipStream_t st) {
    k_guard<<<1, 64, 0, st>>>(g, tol);
    return hipGetLastError();
}

hipError_t launch_moments_final(const double* partials, int nblk, double vol, double c, double s, const double* tp,
                                double Om, double* out, hipStream_t st) {
    k_moments_final<<<1, RED_THREADS, 0, st>>>(partials, nblk, vol, c, s, tp, Om, out);
    return hipGetLastError();
}

hipError_t launch_renorm_factor(const double* partials, int nblk, double vol, double mscale, double* r,
                                hipStream_t st) {
    k_renorm_factor<<<1, RED_THREADS, 0, st>>>(partials, nblk, vol, mscale, r);
    return hipGetLastError();
}

hipError_t launch_time_add(double* t, double dtot, hipStream_t st) {
    k_time_add<<<1, 64, 0, st>>>(t, dtot);
    return hipGetLastError();
}

}  // namespace fse
