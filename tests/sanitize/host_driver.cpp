// Runs the host-side calls of the library (quantizers, length model, FASTA
// parser, Alg. 1 packer, score conversions, plan lookups and the argument
// checks of the device calls that fail before any device work) on random
// and edge inputs.  Built from the library's host source with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code by
// tests/test_sanitizers.py; no GPU is touched.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "hmsv.h"

static int fails = 0;
#define EXPECT(c)                                                   \
    do {                                                            \
        if (!(c)) {                                                 \
            std::fprintf(stderr, "expectation failed: %s\n", #c);   \
            ++fails;                                                \
        }                                                           \
    } while (0)

int main() {
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::vector<double> bg(20);
    for (auto &b : bg) b = 0.02 + u(rng) * 0.05;
    for (int M : {1, 2, 30, 400, 2815}) {
        std::vector<double> e((size_t)M * 20), t((size_t)M * 7);
        for (auto &v : e) v = u(rng) < 0.05 ? 0.0 : u(rng);
        for (auto &v : t) v = u(rng) < 0.05 ? 0.0 : u(rng);
        std::vector<uint8_t> cost((size_t)32 * M);
        std::vector<int8_t> sc((size_t)32 * M);
        int32_t dbias = 0, tbm = 0;
        EXPECT(hmsv_quantize(e.data(), bg.data(), M, cost.data(), sc.data(), &dbias) == HMSV_OK);
        std::vector<int16_t> msc((size_t)32 * M), tr((size_t)7 * M);
        EXPECT(hmsv_p7_quantize(e.data(), t.data(), bg.data(), M, msc.data(), tr.data(), &tbm) ==
               HMSV_OK);
        // (no kernels are linked here: the plan calls may answer
        // HMSV_ENOKERNEL; they run for their host code only)
        hmsv_plan plan;
        (void)hmsv_default_plan(1, M, &plan);
        (void)hmsv_default_plan(0, M, &plan);
        (void)hmsv_p7_default_plan(M, &plan);
        (void)hmsv_tbm(M);
    }
    EXPECT(hmsv_quantize(nullptr, bg.data(), 5, nullptr, nullptr, nullptr) == HMSV_EINVAL);
    for (int64_t L : {(int64_t)0, (int64_t)1, (int64_t)350, (int64_t)100000}) {
        int32_t loop = 0, move = 0;
        EXPECT(hmsv_p7_length_model(L, &loop, &move) == HMSV_OK);
        (void)hmsv_tjb(L);
    }
    for (int G = 1; G <= 64; G *= 2)
        for (int Q = 1; Q <= 32; ++Q) {
            (void)hmsv_plan_lds_bytes(G, Q);
            (void)hmsv_p7_lds_bytes(G, Q);
        }
    (void)hmsv_workspace_bytes(0);
    (void)hmsv_workspace_bytes(1 << 20);

    // FASTA: valid text, then a bad byte, then text with no trailing newline
    const std::string texts[] = {
        ">a one\nACDEFGHIKLMNPQRSTVWY\nbjzuox\n>b\n\n>c\r\nAC-D.E*12\r\n",
        ">a\nAC!D\n", ">x\nMKV", "", ">only header"};
    for (const std::string &s : texts) {
        int64_t nres = 0, nseq = 0, err = 0;
        hmsv_status st = hmsv_fasta_parse(s.data(), (int64_t)s.size(), nullptr, nullptr,
                                          nullptr, &nres, &nseq, &err);
        if (st != HMSV_OK) continue;
        std::vector<uint8_t> res((size_t)(nres > 0 ? nres : 1));
        std::vector<int64_t> off((size_t)nseq + 1), names((size_t)(2 * nseq + 1));
        EXPECT(hmsv_fasta_parse(s.data(), (int64_t)s.size(), res.data(), off.data(),
                                names.data(), &nres, &nseq, &err) == HMSV_OK);
    }

    // Alg. 1 packer on lognormal-like lengths, with and without heights
    std::lognormal_distribution<double> ln(5.58, 0.74);
    std::vector<int64_t> lens(3000);
    for (auto &l : lens) l = (int64_t)std::lround(ln(rng));
    lens[5] = 0;
    std::vector<int32_t> cont(lens.size());
    for (int nb : {1, 7, 480}) {
        std::vector<int64_t> heights((size_t)nb);
        hmsv_alg1_stats st;
        EXPECT(hmsv_alg1_pack(lens.data(), (int64_t)lens.size(), nb, 128, cont.data(),
                              heights.data(), &st) == HMSV_OK);
        EXPECT(hmsv_alg1_pack(lens.data(), (int64_t)lens.size(), nb, 3, cont.data(), nullptr,
                              &st) == HMSV_OK);
    }

    // scores to nats and P-values
    const int64_t n = 256;
    std::vector<uint8_t> sc8((size_t)n), fl((size_t)n);
    std::vector<int64_t> L((size_t)n);
    std::vector<double> nats((size_t)n), p((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        sc8[(size_t)i] = (uint8_t)i;
        fl[(size_t)i] = (uint8_t)(i % 17 == 0);
        L[(size_t)i] = i * 3;
    }
    for (int is_msv = 0; is_msv < 2; ++is_msv) {
        EXPECT(hmsv_score_nats(is_msv, 400, sc8.data(), fl.data(), L.data(), n, nats.data()) ==
               HMSV_OK);
        EXPECT(hmsv_gumbel_pvalue(nats.data(), n, -2.0, 0.7, p.data()) == HMSV_OK);
    }

    // device calls refuse bad arguments before touching a device
    hmsv_profile prof{};
    EXPECT(hmsv_msv_score(&prof, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
           HMSV_EINVAL);
    hmsv_p7_profile p7{};
    EXPECT(hmsv_p7_score(&p7, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
           HMSV_EINVAL);
    EXPECT(hmsv_select(nullptr, nullptr, nullptr, 1, 0, nullptr, nullptr, nullptr, nullptr) ==
           HMSV_EINVAL);
    for (int s = 0; s >= -6; --s) (void)hmsv_strerror(s);
    if (fails) return 1;
    std::puts("host driver done");
    return 0;
}
