// Internal declarations shared by the library's translation units.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "leja_logdet.h"

namespace ld {

// ---- error reporting --------------------------------------------------------
int fail(int code, const std::string& detail);   // sets the thread-local detail, returns code
void clear_error();

// ---- host mathematics (host_math.cpp) ---------------------------------------
// Fast Léja table on [-2, 2], cached and grown on demand; returns a copy of
// the first `count` points (safe against concurrent growth of the table).
std::vector<double> leja_table(int count);

// Alg. 1 divided differences, cached by (lo, hi, degree, s-mode, cap).
int divided_differences(double lo, double hi, int degree, int s_mode, int64_t cap,
                        std::vector<double>& d, int64_t* terms);

// Newton coefficients -> coefficients in the squared basis (pi_a^2, pi_a pi_{a+1}).
void squared_basis(const std::vector<double>& xi, const std::vector<double>& d,
                   std::vector<double>& c);

// SplitMix64 pieces (published generator, Steele-Lea-Flood 2014).
uint64_t splitmix_mix(uint64_t z);
uint64_t probe_stream_key(uint64_t seed, int stream);

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal a[0..k)
// and off-diagonal b[0..k-1) (cyclic Jacobi on the dense k x k matrix), and
// the last component of its unit eigenvector.
void tridiag_top_eigenpair(const std::vector<double>& a, const std::vector<double>& b, double* theta,
                           double* last);

// Neumaier-compensated FP64 sum.
struct KahanSum {
    double s = 0.0, c = 0.0;
    void add(double x);
    double value() const { return s + c; }
};

// Scalars of the mapped recurrence (Sec. 4 scaling + Sec. 3.1 map).
struct Plan {
    double sigma, lo, hi, c, gamma, alpha;
    int degree;
    std::vector<double> xi;    // degree+1 Léja points
    std::vector<double> d;     // degree+1 divided differences
    std::vector<double> beta;  // degree: c/gamma + xi_j
    int64_t taylor_terms;
};
int make_plan(double lmin, double lmax, int degree, const ld_options& o, Plan& p);

}  // namespace ld
