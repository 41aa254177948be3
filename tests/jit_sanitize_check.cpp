// Drives the host-only entry points of the library (expression parser and
// kernel-source generator, size queries, error reporting) with valid,
// malformed and pseudo-random expressions, so that a build of the library's
// host code with AddressSanitizer and UndefinedBehaviorSanitizer can report
// any out-of-bounds access, leak or undefined operation.  Needs no GPU.
// Prints "ok" when every fixed expression is accepted or refused as
// expected.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../include/qdpx.h"

static int generate_all_formats(const std::string &e, int &accepted) {
    int ok = 0;
    char small[64];
    for (int f = 0; f < 3; ++f) {
        const qdpx_prec p = f == 0 ? QDPX_F64 : QDPX_F32;
        const qdpx_linkfmt l = f == 2 ? QDPX_LINK12 : QDPX_LINK18;
        size_t need = 0;
        if (qdpx_jit_generate(e.c_str(), p, l, 2, 1, nullptr, 0, &need) != QDPX_OK) continue;
        std::string s(need, '\0');
        if (qdpx_jit_generate(e.c_str(), p, l, 2, 1, &s[0], need, nullptr) != QDPX_OK) return -1;
        if (s.find("qdpx_jit_kernel") == std::string::npos) return -1;
        if (qdpx_jit_generate(e.c_str(), p, l, 2, 1, small, sizeof small, nullptr) != QDPX_ENOMEM &&
            need > sizeof small)
            return -1;
        ++ok;
        ++accepted;
    }
    return ok;
}

int main() {
    const char *valid[] = {
        "(sum 0xF (add (umul m (shift f0 + m)) (shift (uadj m f0) - m)))",
        "(add f1 (scale s0 (sum 0xF (add (umul m (shift f0 + m)) (shift (uadj m f0) - m)))))",
        "(sub (umul 1 (shift f0 + 1)) (scale s0 (uadj 2 f1)))",
        "f0",
        "(shift (shift f0 + 2) - 2)",
        "(sum 0x7 (umul m (shift f0 + m)))",
        "(add f0 (add f0 (add f0 (add f0 (add f0 (add f0 (add f0 (add f0 f0))))))))",
    };
    const char *invalid[] = {"(add f0 f1", "(umul m f0)", "(sum 0xF (sum 0xF f0))", "((((", ")", "",
                             "(scale s9 f0)", "(add f0 f7)", "(shift f0 * 1)", "(umul 4 f0)", "(sum 0x1F f0)",
                             "(sum zz f0)", "(add f0 f1) f2", "(add f0 99999999999999999999)"};
    int fails = 0, accepted = 0;
    for (const char *e : valid)
        if (generate_all_formats(e, accepted) != 3) {
            std::printf("FAIL valid: %s\n", e);
            ++fails;
        }
    for (const char *e : invalid)
        if (generate_all_formats(e, accepted) != 0) {
            std::printf("FAIL invalid accepted: %s\n", e);
            ++fails;
        }
    // token soup from a fixed xorshift sequence: only the absence of
    // sanitizer reports matters here
    const char *toks[] = {"(", ")", "add", "sub", "scale", "umul", "uadj", "shift", "sum", "f0", "f1", "s0",
                          "m", "0", "3", "+", "-", "0xF", "0x0", "xyz", "99999999999999999999"};
    const int ntok = sizeof toks / sizeof toks[0];
    uint32_t x = 2463534242u;
    for (int i = 0; i < 3000; ++i) {
        std::string e;
        x ^= x << 13, x ^= x >> 17, x ^= x << 5;
        const int n = 1 + (int)(x % 25);
        for (int k = 0; k < n; ++k) {
            x ^= x << 13, x ^= x >> 17, x ^= x << 5;
            e += std::string(toks[x % ntok]) + " ";
        }
        if (generate_all_formats(e, accepted) < 0) {
            std::printf("FAIL generator: %s\n", e.c_str());
            ++fails;
        }
    }
    if (qdpx_jit_generate(nullptr, QDPX_F64, QDPX_LINK18, 1, 0, nullptr, 0, nullptr) != QDPX_EINVAL) ++fails;
    if (qdpx_jit_generate("f0", QDPX_F64, QDPX_LINK12, 1, 0, nullptr, 0, nullptr) != QDPX_EUNSUPPORTED) ++fails;
    const qdpx_geom g{{4, 4, 4, 4}}, bad{{1, 4, 4, 4}};
    if (qdpx_links_bytes(&g, QDPX_F32, QDPX_LINK12) == 0 || qdpx_links_bytes(&bad, QDPX_F64, QDPX_LINK18) != 0) ++fails;
    if (qdpx_eval_hop(nullptr, &g, QDPX_F64, QDPX_LINK18, nullptr, nullptr, nullptr, 0xF, nullptr) != QDPX_EINVAL)
        ++fails;
    if (!fails) std::printf("ok (%d accepted)\n", accepted);
    return fails != 0;
}
