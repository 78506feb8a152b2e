// Several host threads call the Léja table, Alg. 1 and the squared-basis
// coefficients at once, with degrees that make the shared Léja table grow
// while other threads read it.  Built with ThreadSanitizer and, separately,
// with AddressSanitizer by tests/test_host_sanitizers.py; every result is
// compared with the same call made afterwards on one thread.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <thread>
#include <vector>

#include "leja_logdet.h"

namespace {

constexpr int kThreads = 8;
constexpr int kRounds = 6;

// degree asked for by thread t in round r: every round crosses a new
// power-of-two table size, and the threads ask for sizes on both sides of it
int degree_of(int t, int r) { return (32 << r) + (t % 2 ? 7 * t : -3 * t); }

struct Result {
    std::vector<double> xi, d, c;
    int rc = 0;
};

Result run_one(int degree) {
    Result res;
    res.xi.assign(degree + 1, 0.0);
    res.d.assign(degree + 1, 0.0);
    res.c.assign(degree + 1, 0.0);
    res.rc |= ld_leja_points(degree + 1, res.xi.data());
    res.rc |= ld_divided_differences(0.5, 8.5 + degree * 1e-3, degree, LD_SVAL_CENTER, 0, res.d.data(), nullptr);
    res.rc |= ld_squared_basis_coefficients(degree, res.d.data(), res.c.data());
    return res;
}

}  // namespace

int main() {
    std::vector<std::vector<Result>> got(kThreads, std::vector<Result>(kRounds));
    std::atomic<int> ready{0};
    std::vector<std::thread> pool;
    for (int t = 0; t < kThreads; ++t)
        pool.emplace_back([&, t] {
            ready.fetch_add(1);
            while (ready.load() < kThreads) {
            }
            for (int r = 0; r < kRounds; ++r) got[t][r] = run_one(degree_of(t, r));
        });
    for (auto& th : pool) th.join();
    int failures = 0;
    for (int t = 0; t < kThreads; ++t)
        for (int r = 0; r < kRounds; ++r) {
            const Result want = run_one(degree_of(t, r));
            const Result& have = got[t][r];
            if (have.rc != 0 || have.xi != want.xi || have.d != want.d || have.c != want.c) {
                std::printf("FAIL: thread %d round %d degree %d\n", t, r, degree_of(t, r));
                ++failures;
            }
        }
    std::printf(failures ? "thread checks failed\n" : "thread checks passed\n");
    return failures ? 1 : 0;
}
