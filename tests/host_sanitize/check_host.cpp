// Host-side checks of libfse's C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py: argument
// validation (fse_plan_check) over valid and invalid problems, the host FP64
// GauSum multiplier (fse_gausum_symbol_host) for every kernel kind, error
// messages, and the device entry points' failure without a GPU.  Any memory
// error or undefined behaviour aborts the program; a wrong status code makes
// it exit with 1.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fse.h"

static int g_fail = 0;

static void expect(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, fse_last_error());
        g_fail = 1;
    }
}

static fse_kernel kernel(int kind, double mu, double c, double nx, double ny, double nz) {
    fse_kernel k{};
    k.kind = kind;
    k.mu = mu;
    k.prefactor = c;
    k.n[0] = nx;
    k.n[1] = ny;
    k.n[2] = nz;
    return k;
}

int main() {
    const double pi = 3.14159265358979323846;
    const int N2[2] = {64, 48}, N3[3] = {32, 24, 16};
    const double L2[2] = {8.0, 6.0}, L3[3] = {6.0, 5.0, 4.0}, g[3] = {1.0, 1.2, 2.0};
    fse_kernel coul = kernel(FSE_K_COULOMB, 1.0, 1.0 / (2.0 * pi), 0, 0, 1);
    expect(fse_plan_check(2, N2, L2, 0.75, 0.5, g, 100, 1, &coul, FSE_C128) == FSE_OK, "2D Coulomb accepted");
    expect(fse_plan_check(2, N2, L2, 0.75, 0.5, g, 100, 1, nullptr, FSE_C64) == FSE_OK, "no kernel accepted");
    expect(fse_plan_check(4, N2, L2, 0.75, 0.5, g, 100, 1, &coul, FSE_C128) == FSE_ERR_ARG, "d = 4 refused");
    expect(fse_plan_check(2, nullptr, L2, 0.75, 0.5, g, 100, 1, &coul, FSE_C128) == FSE_ERR_ARG, "NULL N refused");
    expect(fse_plan_check(2, N2, nullptr, 0.75, 0.5, g, 100, 1, &coul, FSE_C128) == FSE_ERR_ARG, "NULL L refused");
    expect(fse_plan_check(2, N2, L2, 0.75, 0.5, nullptr, 100, 1, &coul, FSE_C128) == FSE_ERR_ARG, "NULL gamma refused");
    const int bad_sizes[][2] = {{62, 64}, {8, 64}, {1024, 64}, {0, 64}, {-64, 64}, {15, 64}, {64, 70}, {2147483646, 64}};
    for (const auto& n : bad_sizes) expect(fse_plan_check(2, n, L2, 0.75, 0.5, g, 100, 1, &coul, 0) == FSE_ERR_ARG, "size");
    const double nan = std::nan(""), inf = INFINITY;
    const double badL[2] = {8.0, nan};
    expect(fse_plan_check(2, N2, badL, 0.75, 0.5, g, 100, 1, &coul, 0) == FSE_ERR_ARG, "NaN L refused");
    expect(fse_plan_check(2, N2, L2, nan, 0.5, g, 100, 1, &coul, 0) == FSE_ERR_ARG, "NaN s refused");
    expect(fse_plan_check(2, N2, L2, -1.0, 0.5, g, 100, 1, &coul, 0) == FSE_ERR_ARG, "s < 0 refused");
    expect(fse_plan_check(2, N2, L2, 0.75, inf, g, 100, 1, &coul, 0) == FSE_ERR_ARG, "infinite Omega refused");
    expect(fse_plan_check(2, N2, L2, 0.75, 0.5, g, 100, 1, &coul, 7) == FSE_ERR_ARG, "precision 7 refused");
    fse_kernel mu2 = kernel(FSE_K_COULOMB, 1.5, 1.0, 0, 0, 1);
    expect(fse_plan_check(2, N2, L2, 0.75, 0.5, g, 100, 1, &mu2, 0) == FSE_ERR_ARG, "mu > d - 1 refused");
    fse_kernel ddi3 = kernel(FSE_K_DDI3, 1.0, 1.0, 0, 0, 1);
    expect(fse_plan_check(2, N2, L2, 0.75, 0.5, g, 100, 1, &ddi3, 0) == FSE_ERR_ARG, "3D dipole in 2D refused");
    expect(fse_plan_check(3, N3, L3, 0.8, 0.7, g, 200, 50, &ddi3, 0) == FSE_OK, "3D dipole accepted");
    fse_kernel notunit = kernel(FSE_K_DDI3, 1.0, 1.0, 0.5, 0, 0.5);
    expect(fse_plan_check(3, N3, L3, 0.8, 0.7, g, 200, 50, &notunit, 0) == FSE_ERR_ARG, "non-unit axis refused");
    fse_kernel kind9 = kernel(9, 1.0, 1.0, 0, 0, 1);
    expect(fse_plan_check(2, N2, L2, 0.75, 0.5, g, 100, 1, &kind9, 0) == FSE_ERR_ARG, "unknown kind refused");
    expect(std::strlen(fse_last_error()) > 0, "error message set");
    expect(std::strstr(fse_version(), "gfx950") != nullptr, "version string");

    // host multiplier for every kind, on the non-negative octant
    struct Case {
        int d;
        const int* N;
        const double* L;
        fse_kernel k;
    } cases[] = {{2, N2, L2, coul},
                 {3, N3, L3, kernel(FSE_K_COULOMB, 1.0, 1.0 / (4.0 * pi), 0, 0, 1)},
                 {2, N2, L2, kernel(FSE_K_COULOMB, 0.5, 1.0, 0, 0, 1)},
                 {3, N3, L3, ddi3},
                 {3, N3, L3, kernel(FSE_K_DDI3, 1.0, 1.0, 1, 0, 0)},
                 {2, N2, L2, kernel(FSE_K_DDI2, 1.0, 1.0, 0, 0, 1)},
                 {2, N2, L2, kernel(FSE_K_DDI2, 1.0, 1.0, 0.6, 0, 0.8)}};
    for (const Case& c : cases) {
        size_t n = 1;
        for (int j = 0; j < c.d; ++j) n *= (size_t)(c.N[j] + 1);
        std::vector<double> K(n, nan);
        expect(fse_gausum_symbol_host(c.d, c.N, c.L, &c.k, K.data()) == FSE_OK, "symbol computed");
        bool finite = true;
        for (double v : K) finite = finite && std::isfinite(v);
        expect(finite, "symbol finite");
        if (c.k.kind == FSE_K_DDI3) expect(std::fabs(K[0] + 1.0) < 1e-15, "3D dipole symbol -1 at kappa = 0");
        if (c.k.kind == FSE_K_DDI2) expect(K[0] == 0.0, "2D dipole symbol 0 at kappa = 0");
    }
    fse_kernel tilted = kernel(FSE_K_DDI3, 1.0, 1.0, 0.6, 0.8, 0.0);
    std::vector<double> K(33 * 25 * 17);
    expect(fse_gausum_symbol_host(3, N3, L3, &tilted, K.data()) == FSE_ERR_UNSUPPORTED, "tilted axis has no table");
    expect(fse_gausum_symbol_host(3, N3, L3, nullptr, K.data()) == FSE_ERR_ARG, "NULL kernel refused");
    fse_kernel none = kernel(FSE_K_NONE, 1.0, 1.0, 0, 0, 1);
    expect(fse_gausum_symbol_host(3, N3, L3, &none, K.data()) == FSE_ERR_ARG, "no kernel refused");

    // device entry points without a device: a clean status, no plan
    fse_plan p = nullptr;
    const fse_status st = fse_plan_create(&p, 2, N2, L2, 0.75, 0.5, g, 100, 1, &coul, FSE_C128, 0.0, nullptr);
    expect(st == FSE_ERR_HIP || st == FSE_OK, "plan creation status");
    if (st == FSE_OK) fse_plan_destroy(p);
    else expect(p == nullptr, "no plan on failure");
    expect(fse_plan_create(nullptr, 2, N2, L2, 0.75, 0.5, g, 100, 1, &coul, 0, 0.0, nullptr) == FSE_ERR_ARG, "NULL out");
    expect(fse_step(nullptr, nullptr, 1, 1e-3, nullptr) == FSE_ERR_ARG, "NULL plan refused");
    expect(fse_plan_destroy(nullptr) == FSE_OK, "destroy of NULL");
    std::printf(g_fail ? "host checks FAILED\n" : "host checks passed\n");
    return g_fail;
}
