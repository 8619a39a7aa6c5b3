// Drives the host half of the C ABI (ranges, amounts, orders, comparison
// models) under AddressSanitizer and UndefinedBehaviorSanitizer: every entry
// point on valid and invalid arguments, 3-D to 6-D, ragged process counts,
// the row-split regime and both ownership readings.  Exits non-zero on the
// first unexpected status; the sanitizers abort on any finding.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/fftrw.h"

static int failures = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "unexpected: %s (%s)\n", what, fft_last_error());
        ++failures;
    }
}

static std::vector<int8_t> identity_order(int M)
{
    // the first order of the canonical enumeration
    std::vector<int8_t> o((size_t)(M * M));
    expect(fft_order_at(M, 0, o.data()) == FFTRW_OK, "order_at 0");
    return o;
}

int main()
{
    const int64_t shapes[][6] = {{8, 8, 8}, {6, 5, 4}, {4, 6, 5, 3}, {3, 4, 5, 2, 3}, {2, 3, 2, 2, 3, 2}};
    const int ms[] = {3, 3, 4, 5, 6};
    const int64_t ps[] = {1, 2, 3, 7, 20, 48, 100};
    for (int s = 0; s < 5; ++s) {
        const int M = ms[s];
        const int64_t *dims = shapes[s];
        int64_t T = 1;
        for (int i = 0; i < M; ++i) T *= dims[i];
        const int64_t n = fft_order_count(M);
        for (int64_t P : ps) {
            if (P > T) continue;
            // ranges of every process in the natural decomposition
            int8_t perm[6];
            for (int i = 0; i < M; ++i) perm[i] = (int8_t)(M - 1 - i);
            int64_t last_end = -1;
            for (int64_t p = 0; p < P; ++p) {
                int level = 0;
                int64_t xs = 0, xe = 0, st[6], en[6];
                expect(fft_decomp(M, dims, P, perm, p, &level, &xs, &xe, st, en) == FFTRW_OK, "decomp");
                expect(xs == last_end + 1, "ranges consecutive");
                last_end = xe;
            }
            expect(last_end == T - 1, "ranges cover the array");
            // a few orders: amounts, split-row amounts, index round trip
            for (int64_t idx : {(int64_t)0, n / 3, n - 1}) {
                std::vector<int8_t> o((size_t)(M * M));
                expect(fft_order_at(M, idx, o.data()) == FFTRW_OK, "order_at");
                int64_t back = -1;
                expect(fft_order_index(M, o.data(), &back) == FFTRW_OK && back == idx, "order_index");
                std::vector<int64_t> per((size_t)M);
                int64_t tot = 0, ret = 0;
                for (int own : {FFTRW_OWN_LITERAL, FFTRW_OWN_MATCHED}) {
                    const int rc = fft_comm_volume(M, dims, P, o.data(), own, per.data(), &tot, &ret);
                    expect(rc == FFTRW_OK || rc == FFTRW_E_ROWSPLIT, "comm_volume");
                }
                expect(fft_rowsplit_volume(M, dims, P, o.data(), per.data(), &tot) == FFTRW_OK, "rowsplit_volume");
            }
            int64_t bi, bv, nb, wi, wv, nw;
            std::vector<int8_t> bo((size_t)(M * M)), wo((size_t)(M * M));
            expect(fft_order_search(M, dims, P, FFTRW_OWN_LITERAL, &bi, &bv, &nb, &wi, &wv, &nw, bo.data(),
                                    wo.data()) == FFTRW_OK && bv <= wv && nb >= 1,
                   "order_search");
            if (M <= 4) {
                std::vector<int64_t> vols((size_t)n);
                expect(fft_order_volumes(M, dims, P, FFTRW_OWN_LITERAL, vols.data()) == FFTRW_OK &&
                           vols[(size_t)bi] == bv,
                       "order_volumes");
            }
            if (M <= 5 && P <= 48) {
                int64_t f = 1;
                for (int i = 2; i <= M; ++i) f *= i;
                std::vector<int64_t> tab((size_t)(f * f));
                expect(fft_transpose_volumes(M, dims, P, FFTRW_OWN_MATCHED, tab.data()) == FFTRW_OK,
                       "transpose_volumes");
                std::vector<int64_t> C((size_t)(P * P));
                std::vector<int8_t> id = identity_order(M);
                expect(fft_pair_counts(M, dims, P, id.data(), id.data() + M, C.data()) == FFTRW_OK, "pair_counts");
            }
        }
    }
    // invalid arguments
    const int64_t d3[3] = {4, 4, 4}, d0[3] = {4, 0, 4}, d7[7] = {2, 2, 2, 2, 2, 2, 2};
    int level;
    int64_t xs, xe, tot;
    const int8_t id3[3] = {0, 1, 2};
    expect(fft_decomp(7, d7, 2, id3, 0, &level, &xs, &xe, nullptr, nullptr) == FFTRW_E_SIZE, "M = 7");
    expect(fft_decomp(3, d0, 2, id3, 0, &level, &xs, &xe, nullptr, nullptr) == FFTRW_E_SIZE, "size 0");
    expect(fft_decomp(3, d3, 0, id3, 0, &level, &xs, &xe, nullptr, nullptr) == FFTRW_E_ARG, "P = 0");
    expect(fft_decomp(3, d3, 65, id3, 0, &level, &xs, &xe, nullptr, nullptr) == FFTRW_E_ROWSPLIT, "P > T");
    const int8_t bad[9] = {0, 1, 2, 0, 1, 2, 1, 2, 0};
    expect(fft_comm_volume(3, d3, 4, bad, FFTRW_OWN_LITERAL, nullptr, &tot, nullptr) == FFTRW_E_ORDER, "bad order");
    expect(fft_comm_volume(3, d3, 4, nullptr, FFTRW_OWN_LITERAL, nullptr, &tot, nullptr) != FFTRW_OK, "null order");
    double models[5];
    expect(fft_compare_models(64, 4096, models) == FFTRW_OK && models[0] > 0, "compare_models");
    expect(fft_compare_models(64, 0, models) == FFTRW_E_ARG, "compare_models P = 0");
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
