// CPU-only harness of the library's host logic, built with address and
// undefined-behaviour sanitizers: the history fit (Brent's method on the
// Appendix-A equation), table geometry, the inversion and growth tables, the
// workspace layout of every grid size, and the host argument checks of the
// compute calls (which return before touching a device).  Prints one line per
// group and exits non-zero on the first failed expectation.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2109_10375_amd/csrc/internal.h"

static int fails = 0;
#define EXPECT(c)                                                      \
    do {                                                               \
        if (!(c)) {                                                    \
            std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                                   \
        }                                                              \
    } while (0)

int main() {
    // 1. history fits over the parameter box the batched workloads draw from, and beyond
    int fitted = 0, rejected = 0;
    for (double zm = 6.0; zm <= 10.0; zm += 1.0)
        for (double dz = 0.5; dz <= 8.0; dz += 1.5)
            for (double az = 0.3; az <= 16.0; az *= 1.6) {
                amber_history h{zm, dz, az, 0.0, 0.0, 0.0};
                amber_weibull w{};
                const int rc = amber_weibull_fit(&h, &w);
                if (rc == AMBER_OK) {
                    ++fitted;
                    EXPECT(w.a_w > 0 && w.b_w > 0 && w.c_w > 0 && w.h > 0 && w.z_top > w.a_w);
                    EXPECT(w.table_n > (1 << 21) && w.table_n <= (1 << 22) + 1);
                    // the fitted curve passes the three points of Sec. 3.1.1
                    const double z_ear = zm + dz * az / (1 + az), z_lat = z_ear - dz;
                    const double xs[3] = {0.05, 0.5, 0.95}, zs[3] = {z_ear, zm, z_lat};
                    for (int k = 0; k < 3; ++k) {
                        const double x = std::exp(-std::pow((zs[k] - w.a_w) / w.b_w, w.c_w));
                        EXPECT(std::fabs(x - xs[k]) < 1e-9);
                    }
                } else {
                    ++rejected;
                    EXPECT(rc == AMBER_E_HISTORY);
                }
            }
    std::printf("fits: %d fitted, %d rejected\n", fitted, rejected);

    // 2. argument errors
    amber_history bad{8.0, -1.0, 3.0, 0, 0, 0};
    amber_weibull w{};
    EXPECT(amber_weibull_fit(&bad, &w) == AMBER_E_ARG);
    EXPECT(amber_weibull_fit(nullptr, &w) == AMBER_E_ARG);
    EXPECT(amber_weibull_from_coeffs(-1.0, 1.0, 1.0, &w) == AMBER_E_HISTORY);
    EXPECT(amber_weibull_from_coeffs(6.9, 1.5, NAN, &w) == AMBER_E_HISTORY);

    // 3. tables: exact sizes, monotone values (written into exactly table_n slots)
    amber_history fid{8.0, 4.0, 3.0, 0, 0, 0};
    EXPECT(amber_weibull_fit(&fid, &w) == AMBER_OK);
    std::vector<double> X((size_t)w.table_n), XG(2 * (size_t)w.table_n);
    EXPECT(amber_weibull_table(&w, X.data(), w.table_n - 1) == AMBER_E_ARG);
    EXPECT(amber_weibull_table(&w, X.data(), w.table_n) == AMBER_OK);
    EXPECT(X[0] == 1.0);
    for (size_t j = 1; j < X.size(); ++j) EXPECT(X[j] <= X[j - 1]);
    EXPECT(amber_growth_table(&w, 8.0, 0.3, XG.data(), w.table_n) == AMBER_OK);
    EXPECT(amber_growth_table(&w, 8.0, 1.5, XG.data(), w.table_n) == AMBER_E_ARG);
    for (size_t j = 1; j < X.size(); ++j) EXPECT(XG[2 * j] == X[j] && XG[2 * j + 1] < XG[2 * j - 1]);
    amber_weibull q{};
    EXPECT(amber_history_prepare(&fid, &q, nullptr, 0, nullptr) == AMBER_OK);  // size query, no device
    EXPECT(q.table_n == w.table_n && q.d_table == nullptr);
    std::printf("tables: %lld nodes, X_T = %.3e, G_0 = %.6f\n", (long long)w.table_n, X.back(), XG[1]);

    // 4. workspace layout of every supported grid size: regions in bounds and disjoint where they must be
    const int sizes[] = {8, 16, 32, 64, 96, 128, 192, 256, 512, 1024};
    for (int n : sizes)
        for (int nl : {1, 2, 8})
            for (bool halo : {false, true}) {
                const WsLayout L = ws_layout(n, nl, halo);
                const size_t n3 = (size_t)n * n * n;
                EXPECT(L.ctrl == 0 && L.spec_a >= sizeof(Ctrl));
                EXPECT(L.nyq_a + (size_t)n * n * 8 <= L.total);
                EXPECT(L.part2[1] + n3 * 4 <= L.lookback);
                EXPECT(L.lookback + (size_t)lb_words((long long)n3) * 12 <= L.total);
                for (int i = 0; i < 2; ++i) EXPECT(L.keys[i] % 256 == 0 && L.vals[i] % 256 == 0 && L.wts[i] % 256 == 0);
                if (nl > 1) EXPECT(L.spec_b >= L.nyq_a + (size_t)n * n * 8);
                if (halo) EXPECT(L.mesh[1] + n3 * 4 <= L.bins && L.halo_tab + (size_t)n * 32 <= L.total);
            }
    // the no-allocation matching call's static scratch holds the workspace of its largest grid
    EXPECT(ws_layout(AMBER_NOALLOC_MAX_N, 1).total <= (size_t)AMBER_NOALLOC_SCRATCH_BYTES);
    std::printf("layouts: %zu sizes; no-allocation scratch %zu of %zu bytes used at N = %d\n",
                sizeof(sizes) / sizeof(sizes[0]), ws_layout(AMBER_NOALLOC_MAX_N, 1).total,
                (size_t)AMBER_NOALLOC_SCRATCH_BYTES, AMBER_NOALLOC_MAX_N);

    // 5. compute calls reject bad arguments on the host, before any device work
    float* dummy = reinterpret_cast<float*>(X.data());
    float* outs[1] = {dummy};
    EXPECT(amber_radiation(nullptr, dummy, nullptr, 1, outs, dummy, 0, nullptr) == AMBER_E_ARG);
    EXPECT(amber_zre(nullptr, dummy, dummy, &w, 1, outs, dummy, 0, nullptr) == AMBER_E_ARG);
    EXPECT(amber_workspace_bytes(nullptr, 1, 1) == 0);
    EXPECT(amber_batch_workspace_bytes(nullptr, 0, 1) == 0);
    EXPECT(amber_batch_run(nullptr, 1, nullptr, nullptr, 0, nullptr, nullptr) == AMBER_E_ARG);
    amber_executor ex = nullptr;
    EXPECT(amber_executor_create(&ex, 0) == AMBER_E_ARG && ex == nullptr);
    unsigned st = 0;
    EXPECT(amber_status(nullptr, nullptr, &st) == AMBER_E_ARG);
    amber_plan plan = nullptr;
    EXPECT(amber_plan_create(&plan, 100, 1.0) == AMBER_E_SIZE && plan == nullptr);
    std::printf("argument checks done\n");
    if (fails) std::printf("%d expectation(s) failed\n", fails);
    return fails ? 1 : 0;
}
