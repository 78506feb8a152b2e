// Host-side mathematics of the Léja + Hutch++ estimator: Léja points, divided
// differences by the scaled Taylor matrix function (Alg. 1), the change to the
// squared Newton basis, the probe generator, a small Cholesky, and the
// thread-local error detail.  Everything here is FP64 (or double-double)
// scalar work done once per call or cached across calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "ld_internal.h"

namespace ld {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_detail;

int fail(int code, const std::string& detail) {
    g_detail = detail;
    return code;
}
void clear_error() { g_detail.clear(); }

// ---------------------------------------------------------------------------
// Real fast Léja points on [-2, 2] (Sec. 3, Eq. Léja5).  The maximum of
// prod_k |x - xi_k| is searched over the midpoints of adjacent points already
// chosen (the fast Léja algorithm the paper uses).  Each candidate keeps its
// product; when a point is added, the surviving candidates multiply in one
// more factor and the two new midpoints get their full product, so every
// product is formed in index order k = 0, 1, ... as a direct evaluation would.
// Ties (relative 1e-12) go to the larger x.
// ---------------------------------------------------------------------------
namespace {
constexpr double kTieRtol = 1e-12;

struct Cand {
    double x, prod;
};

std::vector<double> compute_leja(int count) {
    std::vector<double> pts;
    if (count <= 0) return pts;
    pts.reserve(count);
    pts.push_back(2.0);
    if (count == 1) return pts;
    pts.push_back(-2.0);
    std::vector<Cand> cands;
    auto full_product = [&](double x) {
        double p = 1.0;
        for (double q : pts) p *= std::fabs(x - q);
        return p;
    };
    cands.push_back({0.0, full_product(0.0)});
    // sorted copy of the chosen points, for finding neighbours
    std::vector<double> sorted = {-2.0, 2.0};
    while ((int)pts.size() < count) {
        double pmax = 0.0;
        for (const Cand& c : cands) pmax = std::fmax(pmax, c.prod);
        int best = -1;
        for (int i = 0; i < (int)cands.size(); ++i) {
            if (cands[i].prod >= pmax * (1.0 - kTieRtol) &&
                (best < 0 || cands[i].x > cands[best].x))
                best = i;
        }
        const double x = cands[best].x;
        cands.erase(cands.begin() + best);
        // neighbours of x among the sorted points
        auto it = std::lower_bound(sorted.begin(), sorted.end(), x);
        const double right = *it, left = *(it - 1);
        sorted.insert(it, x);
        for (Cand& c : cands) c.prod *= std::fabs(c.x - x);
        pts.push_back(x);
        const double m1 = 0.5 * (left + x), m2 = 0.5 * (x + right);
        cands.push_back({m1, full_product(m1)});
        cands.push_back({m2, full_product(m2)});
    }
    return pts;
}
}  // namespace

std::vector<double> leja_table(int count) {
    // The table grows by reassignment; callers get a copy of their prefix,
    // taken under the lock, so a concurrent call that grows the table never
    // frees memory another thread is still reading.
    static std::mutex mu;
    static std::vector<double> table;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)table.size() < count) {
        int want = 64;
        while (want < count) want *= 2;
        table = compute_leja(want);
    }
    return std::vector<double>(table.begin(), table.begin() + std::max(count, 0));
}

// ---------------------------------------------------------------------------
// Alg. 1: d = log(Q_m) e_1 with Q_m = cI + gamma*Q^_m, Q^_m lower bidiagonal
// (Léja points on the diagonal, ones below; Eq. eq_leja_matrix).  With the
// scaling value s, log(Q_m) = log(s) I + log(I + W), W = (Q_m - sI)/s, and the
// Taylor series of log(I + W) is summed term by term on the vector W^k e_1.
// W is lower bidiagonal: (W v)_i = w_ii v_i + (gamma/s) v_{i-1}.
// ---------------------------------------------------------------------------
static int alg1(double lo, double hi, int degree, int s_mode, int64_t cap,
                std::vector<double>& d, int64_t* terms) {
    const std::vector<double> xi_all = leja_table(degree + 1);
    const int m1 = degree + 1;
    const double c = 0.5 * (lo + hi);
    const double gamma = 0.25 * (hi - lo);
    const double s = (s_mode == LD_SVAL_CENTER) ? c : 0.5 * hi;
    std::vector<double> diag(m1), v(m1, 0.0), w(m1), acc(m1, 0.0);
    for (int i = 0; i < m1; ++i) diag[i] = (c + gamma * xi_all[i] - s) / s;
    const double sub = gamma / s;
    v[0] = 1.0;
    acc[0] = std::log(s);
    int64_t p = 0;
    for (int64_t k = 1; k <= cap; ++k) {
        w[0] = diag[0] * v[0];
        for (int i = 1; i < m1; ++i) w[i] = diag[i] * v[i] + sub * v[i - 1];
        const double coef = ((k & 1) ? 1.0 : -1.0) / (double)k;
        double tmax = 0.0, amax = 0.0;
        for (int i = 0; i < m1; ++i) {
            v[i] = w[i];
            const double t = coef * w[i];
            acc[i] += t;
            tmax = std::fmax(tmax, std::fabs(t));
            amax = std::fmax(amax, std::fabs(acc[i]));
        }
        p = k;
        if (k > 10 && tmax <= 0x1p-60 * amax) break;
    }
    d = acc;
    if (terms) *terms = p;
    return LD_OK;
}

int divided_differences(double lo, double hi, int degree, int s_mode, int64_t cap,
                        std::vector<double>& d, int64_t* terms) {
    if (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi) || degree < 0)
        return fail(LD_EINVAL, "divided differences need 0 < lo < hi and degree >= 0");
    if (s_mode != LD_SVAL_CENTER && s_mode != LD_SVAL_HALF_LMAX)
        return fail(LD_EINVAL, "unknown s_val_mode");
    if (cap <= 0) cap = 100000000;
    using Key = std::tuple<double, double, int, int, int64_t>;
    static std::mutex mu;
    static std::map<Key, std::pair<std::vector<double>, int64_t>> cache;
    const Key key{lo, hi, degree, s_mode, cap};
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            d = it->second.first;
            if (terms) *terms = it->second.second;
            return LD_OK;
        }
    }
    int64_t p = 0;
    int rc = alg1(lo, hi, degree, s_mode, cap, d, &p);
    if (rc != LD_OK) return rc;
    if (terms) *terms = p;
    std::lock_guard<std::mutex> lock(mu);
    if (cache.size() > 256) cache.clear();
    cache[key] = {d, p};
    return LD_OK;
}

// ---------------------------------------------------------------------------
// Squared Newton basis.  The products q_2a = pi_a^2 and q_2a+1 = pi_a pi_{a+1}
// are the Newton basis of the doubled centre sequence
// zeta = (xi_0, xi_0, xi_1, xi_1, ...).  A Newton form is moved to new
// centres one at a time: prepending a centre z and dropping the last one maps
// coefficients a to a' with a'_n = a_n, a'_i = a_i + (z - C_i) a'_{i+1}
// (nested multiplication, de Boor, "A Practical Guide to Splines", ch. I).
// Prepending zeta_{m-1}, ..., zeta_0 in turn yields the zeta form.  The O(m^2)
// updates run in double-double arithmetic so that the result is correct to
// FP64 even where the basis change amplifies rounding.
// ---------------------------------------------------------------------------
namespace {
struct DD {
    double hi, lo;
};
inline DD two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
inline DD dd_add(DD a, DD b) {
    DD s = two_sum(a.hi, b.hi);
    DD t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return two_sum(s.hi, s.lo);
}
inline DD dd_mul(DD a, DD b) {
    double p = a.hi * b.hi;
    double e = std::fma(a.hi, b.hi, -p);
    e += a.hi * b.lo + a.lo * b.hi;
    return two_sum(p, e);
}
}  // namespace

void squared_basis(const std::vector<double>& xi, const std::vector<double>& d,
                   std::vector<double>& c) {
    const int n = (int)d.size() - 1;
    std::vector<DD> a(n + 1), ap(n + 1);
    std::vector<double> C(n > 0 ? n : 1);
    for (int i = 0; i <= n; ++i) a[i] = {d[i], 0.0};
    for (int i = 0; i < n; ++i) C[i] = xi[i];
    for (int t = n - 1; t >= 0; --t) {
        const double z = xi[t / 2];
        ap[n] = a[n];
        for (int i = n - 1; i >= 0; --i) {
            DD diff = two_sum(z, -C[i]);
            ap[i] = dd_add(a[i], dd_mul(diff, ap[i + 1]));
        }
        a.swap(ap);
        for (int i = n - 1; i >= 1; --i) C[i] = C[i - 1];
        if (n > 0) C[0] = z;
    }
    c.resize(n + 1);
    for (int i = 0; i <= n; ++i) c[i] = a[i].hi + a[i].lo;
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014; reference code by S. Vigna).
// ---------------------------------------------------------------------------
uint64_t splitmix_mix(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}
uint64_t probe_stream_key(uint64_t seed, int stream) {
    return splitmix_mix(seed + (uint64_t)(stream + 1) * 0x9E3779B97F4A7C15ull);
}

void tridiag_top_eigenpair(const std::vector<double>& a, const std::vector<double>& b, double* theta,
                           double* last) {
    const int k = (int)a.size();
    std::vector<double> M((size_t)k * k, 0.0), V((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) {
        M[(size_t)i * k + i] = a[i];
        V[(size_t)i * k + i] = 1.0;
        if (i + 1 < k) M[(size_t)i * k + i + 1] = M[(size_t)(i + 1) * k + i] = b[i];
    }
    // cyclic Jacobi: rotate away each off-diagonal entry in turn until the
    // off-diagonal mass is negligible against the diagonal
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                const double x = M[(size_t)i * k + j];
                (i == j ? dia : off) += x * x;
            }
        if (off <= 1e-32 * dia || off == 0.0) break;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = M[(size_t)p * k + q];
                if (apq == 0.0) continue;
                const double app = M[(size_t)p * k + p], aqq = M[(size_t)q * k + q];
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < k; ++r) {   // M <- M J (columns p, q)
                    const double mp = M[(size_t)r * k + p], mq = M[(size_t)r * k + q];
                    M[(size_t)r * k + p] = c * mp - s * mq;
                    M[(size_t)r * k + q] = s * mp + c * mq;
                }
                for (int r = 0; r < k; ++r) {   // M <- J^T M (rows p, q)
                    const double mp = M[(size_t)p * k + r], mq = M[(size_t)q * k + r];
                    M[(size_t)p * k + r] = c * mp - s * mq;
                    M[(size_t)q * k + r] = s * mp + c * mq;
                }
                for (int r = 0; r < k; ++r) {   // V <- V J
                    const double vp = V[(size_t)r * k + p], vq = V[(size_t)r * k + q];
                    V[(size_t)r * k + p] = c * vp - s * vq;
                    V[(size_t)r * k + q] = s * vp + c * vq;
                }
            }
    }
    int top = 0;
    for (int i = 1; i < k; ++i)
        if (M[(size_t)i * k + i] > M[(size_t)top * k + top]) top = i;
    *theta = M[(size_t)top * k + top];
    *last = V[(size_t)(k - 1) * k + top];   // column `top` of V is the eigenvector
}

void KahanSum::add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

// ---------------------------------------------------------------------------
// Scaling (Eq. scaled_sigma_matrix, with the input lower bound) and the mapped
// recurrence scalars: T = (Q~ - cI)/gamma = alpha*Q - (c/gamma) I,
// (T - xi_j I) w = alpha*Q w - beta_j w.
// ---------------------------------------------------------------------------
int make_plan(double lmin, double lmax, int degree, const ld_options& o, Plan& p) {
    if (!(lmin > 0.0) || !(lmax > lmin) || !std::isfinite(lmax))
        return fail(LD_EINVAL, "need 0 < lmin < lmax");
    if (degree < 1) return fail(LD_EINVAL, "degree must be >= 1");
    p.degree = degree;
    p.sigma = lmin < 1.0 ? lmin : 1.0;
    p.lo = lmin / p.sigma;
    p.hi = lmax / p.sigma;
    p.c = 0.5 * (p.lo + p.hi);
    p.gamma = 0.25 * (p.hi - p.lo);
    p.alpha = 1.0 / (p.sigma * p.gamma);
    p.xi = leja_table(degree + 1);
    int rc = divided_differences(p.lo, p.hi, degree, o.s_val_mode, o.taylor_cap, p.d,
                                 &p.taylor_terms);
    if (rc != LD_OK) return rc;
    p.beta.resize(degree);
    for (int j = 0; j < degree; ++j) p.beta[j] = p.c / p.gamma + p.xi[j];
    return LD_OK;
}

}  // namespace ld

// ---------------------------------------------------------------------------
// host entry points
// ---------------------------------------------------------------------------
extern "C" {

#ifndef LD_SOURCE_HASH
#define LD_SOURCE_HASH "unknown"
#endif
// "src=" carries the hash of the source files the library was built from
// (computed by the build script), so a run can tell which sources it loaded.
const char* ld_version(void) { return "leja_logdet 0.2 (gfx950) src=" LD_SOURCE_HASH; }

const char* ld_error_string(int code) {
    switch (code) {
        case LD_OK: return "LD_OK";
        case LD_EINVAL: return "LD_EINVAL: invalid argument";
        case LD_ECSR: return "LD_ECSR: invalid CSR structure";
        case LD_EBREAKDOWN: return "LD_EBREAKDOWN: CholQR Gram matrix not positive definite";
        case LD_EWORKSPACE: return "LD_EWORKSPACE: workspace too small";
        case LD_EHIP: return "LD_EHIP: HIP runtime error";
        case LD_EINDEF: return "LD_EINDEF: Gershgorin lower bound is not positive";
        case LD_ENOMEM: return "LD_ENOMEM: allocation failed";
        default: return "unknown error code";
    }
}

const char* ld_last_error_detail(void) { return ld::g_detail.c_str(); }

void ld_default_options(ld_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->s_val_mode = LD_SVAL_CENTER;
    o->dot_mode = LD_DOT_AUTO;
}

int ld_leja_points(int32_t count, double* xi_host) {
    ld::clear_error();
    if (count < 0 || (count > 0 && !xi_host)) return ld::fail(LD_EINVAL, "bad count or null");
    if (count == 0) return LD_OK;
    const std::vector<double> t = ld::leja_table(count);
    std::memcpy(xi_host, t.data(), sizeof(double) * count);
    return LD_OK;
}

int ld_divided_differences(double lo, double hi, int32_t degree, int32_t s_val_mode,
                           int64_t taylor_cap, double* d_host, int64_t* terms) {
    ld::clear_error();
    if (!d_host) return ld::fail(LD_EINVAL, "d_host is null");
    std::vector<double> d;
    int rc = ld::divided_differences(lo, hi, degree, s_val_mode, taylor_cap, d, terms);
    if (rc != LD_OK) return rc;
    std::memcpy(d_host, d.data(), sizeof(double) * (degree + 1));
    return LD_OK;
}

int ld_rademacher_host(uint64_t seed, int32_t stream, int64_t n, int64_t row0, int64_t nrows,
                       int64_t col0, int64_t ncols, int8_t* out_host) {
    ld::clear_error();
    if (n < 0 || row0 < 0 || nrows < 0 || col0 < 0 || ncols < 0 || stream < 0 ||
        (nrows * ncols > 0 && !out_host))
        return ld::fail(LD_EINVAL, "bad probe range");
    const uint64_t key = ld::probe_stream_key(seed, stream);
    for (int64_t r = 0; r < nrows; ++r)
        for (int64_t c = 0; c < ncols; ++c) {
            const uint64_t i = (uint64_t)(col0 + c) * (uint64_t)n + (uint64_t)(row0 + r) + 1;
            const uint64_t x = ld::splitmix_mix(key + i * 0x9E3779B97F4A7C15ull);
            out_host[r * ncols + c] = (x >> 63) ? -1 : 1;
        }
    return LD_OK;
}

int ld_squared_basis_coefficients(int32_t degree, const double* d_host, double* c_host) {
    ld::clear_error();
    if (degree < 0 || !d_host || !c_host) return ld::fail(LD_EINVAL, "bad arguments");
    std::vector<double> d(d_host, d_host + degree + 1), c;
    const std::vector<double> xi = ld::leja_table(degree + 1);
    ld::squared_basis(xi, d, c);
    std::memcpy(c_host, c.data(), sizeof(double) * (degree + 1));
    return LD_OK;
}

}  // extern "C"
