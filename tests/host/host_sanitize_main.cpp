// Drives every host-side entry point of the library (Léja table, Alg. 1,
// squared-basis coefficients, probe generator, error strings, the tridiagonal
// eigen-solver of the Lanczos bound) over ordinary and edge-case arguments.
// Built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py; any memory error or undefined behaviour ends
// the program with a non-zero status.
#include <cmath>
#include <cstdio>
#include <vector>

#include "ld_internal.h"

static int failures = 0;
static void expect(bool ok, const char* what) {
    if (!ok) {
        std::printf("FAIL: %s\n", what);
        ++failures;
    }
}

int main() {
    // Léja points: nested tables of many sizes, and argument errors
    for (int count : {0, 1, 2, 3, 17, 161, 301}) {
        std::vector<double> xi(count > 0 ? count : 1);
        expect(ld_leja_points(count, xi.data()) == LD_OK, "leja_points");
    }
    expect(ld_leja_points(-1, nullptr) == LD_EINVAL, "leja_points negative");
    expect(ld_leja_points(4, nullptr) == LD_EINVAL, "leja_points null");

    // Alg. 1 divided differences: both scaling values, several intervals and
    // degrees, a tiny Taylor cap, invalid intervals
    for (int mode : {LD_SVAL_CENTER, LD_SVAL_HALF_LMAX})
        for (double lo : {0.01, 0.5, 1.0})
            for (int degree : {0, 1, 40, 150}) {
                std::vector<double> d(degree + 1);
                int64_t terms = 0;
                // s = hi/2 sits on the Taylor disc's boundary (order grows like 1/accuracy): capped
                const int64_t cap = mode == LD_SVAL_HALF_LMAX ? 3000 : 0;
                const int rc = ld_divided_differences(lo, lo * 1e3 + 8.0, degree, mode, cap, d.data(), &terms);
                expect(rc == LD_OK, "divided_differences");
                for (double v : d) expect(std::isfinite(v), "finite divided differences");
            }
    {
        std::vector<double> d(31);
        expect(ld_divided_differences(0.5, 8.5, 30, LD_SVAL_CENTER, 5, d.data(), nullptr) == LD_OK, "taylor cap");
        expect(ld_divided_differences(2.0, 1.0, 30, LD_SVAL_CENTER, 0, d.data(), nullptr) == LD_EINVAL, "lo > hi");
        expect(ld_divided_differences(0.0, 1.0, 30, LD_SVAL_CENTER, 0, d.data(), nullptr) == LD_EINVAL, "lo = 0");
        expect(ld_divided_differences(0.5, 8.5, 30, 7, 0, d.data(), nullptr) == LD_EINVAL, "bad s_val_mode");
    }

    // squared-basis coefficients of the Newton polynomial
    for (int degree : {1, 2, 3, 40, 81, 150}) {
        std::vector<double> d(degree + 1), c(2 * ((degree + 1) / 2) + 1);
        ld_divided_differences(0.1, 8.1, degree, LD_SVAL_CENTER, 0, d.data(), nullptr);
        expect(ld_squared_basis_coefficients(degree, d.data(), c.data()) == LD_OK, "squared basis");
    }

    // probe generator: windows of rows and columns, empty windows, errors
    {
        std::vector<int8_t> out(64 * 7);
        expect(ld_rademacher_host(3, 0, 1000, 0, 64, 0, 7, out.data()) == LD_OK, "rademacher");
        expect(ld_rademacher_host(3, 1, 1000, 936, 64, 5, 2, out.data()) == LD_OK, "rademacher tail");
        expect(ld_rademacher_host(3, 1, 1000, 0, 0, 0, 0, out.data()) == LD_OK, "rademacher empty");
        expect(ld_rademacher_host(3, 1, 1000, -1, 4, 0, 1, out.data()) == LD_EINVAL, "rademacher negative");
    }

    // error strings and options
    for (int code = -8; code <= 0; ++code) expect(ld_error_string(code) != nullptr, "error string");
    expect(ld_last_error_detail() != nullptr, "error detail");
    expect(ld_version() != nullptr, "version");
    ld_options o;
    ld_default_options(&o);
    ld_default_options(nullptr);

    // the tridiagonal eigen-solver behind the Lanczos bound
    for (int k : {1, 2, 5, 64, 200}) {
        std::vector<double> a(k), b(k > 1 ? k - 1 : 0);
        for (int i = 0; i < k; ++i) a[i] = 2.0 + 0.01 * i;
        for (size_t i = 0; i < b.size(); ++i) b[i] = -1.0;
        double theta = 0.0, last = 0.0;
        ld::tridiag_top_eigenpair(a, b, &theta, &last);
        expect(std::isfinite(theta) && std::isfinite(last), "tridiagonal eigenpair");
    }

    std::printf(failures ? "host checks failed\n" : "host checks passed\n");
    return failures ? 1 : 0;
}
