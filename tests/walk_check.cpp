// Host check of the kernels' site addressing, compiled from the same header
// the kernels use (its device functions are made host-callable here):
//  * group_site covers every site of the lattice exactly once, and its
//    coordinates agree with the site index and with Site::init;
//  * hop_fwd / hop_bwd give the periodic neighbour x +- mu;
//  * traverse (t window) and slabwalk (XCD slab walk, where the launch takes
//    it) are bijections on the group indices, and so is xcd_tile on blocks;
//  * the link layouts map (mu, element, site) one to one onto the link
//    buffer, and FP32 pairs share one 16-byte-aligned entry.
// Over brick, linear and ragged lattices.  Prints "ok" and the number of
// lattices checked.
#include <hip/hip_runtime.h>
#undef __device__
#define __device__ __attribute__((host)) __attribute__((device))
#include "../paper_1105_2279_amd/csrc/qdpx_impl.hpp"

#include <cstdio>
#include <vector>

using namespace qdpx;

static long fails = 0;

#define EXPECT(cond, ...)                         \
    do {                                          \
        if (!(cond)) {                            \
            if (fails < 10) std::printf(__VA_ARGS__); \
            ++fails;                              \
        }                                         \
    } while (0)

static bool bijection(int n, const std::vector<int> &img) {
    std::vector<char> seen(n, 0);
    for (int v : img) {
        if (v < 0 || v >= n || seen[v]) return false;
        seen[v] = 1;
    }
    return (int)img.size() == n;
}

static void check_lattice(const int32_t L[4]) {
    const Geo g = make_geo(L);
    const int V = L[0] * L[1] * L[2] * L[3];
    const int ng = num_groups(g);
    std::vector<int> count(V, 0);
    for (int grp = 0; grp < ng; ++grp)
        for (int lane = 0; lane < 64; ++lane) {
            Site x;
            if (!group_site(g, grp, lane, x)) continue;
            EXPECT(x.s >= 0 && x.s < V, "site %d out of range\n", x.s);
            if (x.s < 0 || x.s >= V) continue;
            ++count[x.s];
            int idx = 0;
            for (int mu = 3; mu >= 0; --mu) {
                EXPECT(x.c[mu] >= 0 && x.c[mu] < L[mu], "coordinate out of range\n");
                idx = idx * L[mu] + x.c[mu];
            }
            EXPECT(idx == x.s, "coordinates disagree with the index at %d\n", x.s);
            Site y;
            y.init(g, x.s);
            for (int mu = 0; mu < 4; ++mu) {
                EXPECT(y.c[mu] == x.c[mu], "Site::init disagrees at %d\n", x.s);
                int c[4] = {x.c[0], x.c[1], x.c[2], x.c[3]};
                c[mu] = (c[mu] + 1) % L[mu];
                const int f = c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]));
                c[mu] = (x.c[mu] + L[mu] - 1) % L[mu];
                const int b = c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]));
                EXPECT(hop_fwd(g, x.s, coord(x, mu), mu) == f, "hop_fwd wrong at %d mu %d\n", x.s, mu);
                EXPECT(hop_bwd(g, x.s, coord(x, mu), mu) == b, "hop_bwd wrong at %d mu %d\n", x.s, mu);
            }
        }
    for (int s = 0; s < V; ++s) EXPECT(count[s] == 1, "site %d covered %d times\n", s, count[s]);
    for (int tw = 1; tw <= 16; tw *= 2) {
        if (L[3] % tw) continue;
        std::vector<int> img(ng);
        for (int i = 0; i < ng; ++i) img[i] = traverse(g, i, tw);
        EXPECT(bijection(ng, img), "traverse tw %d not a bijection on %dx%dx%dx%d\n", tw, L[0], L[1], L[2], L[3]);
    }
    for (int m = 1; m <= 16; m *= 2) {
        LaunchCfg cfg;
        cfg.xcd = 2;
        if (launch_order(g, cfg, m) != 2) continue;
        std::vector<int> img(ng);
        for (int i = 0; i < ng; ++i) img[i] = slabwalk(g, i, m);
        EXPECT(bijection(ng, img), "slabwalk m %d not a bijection on %dx%dx%dx%d\n", m, L[0], L[1], L[2], L[3]);
    }
}

template <typename R, int NR> static void check_layout(int64_t S) {
    using Lay = LinkLayout<R, NR>;
    const int64_t n = 4 * 3 * NR * S;
    std::vector<char> seen(n, 0);
    for (int mu = 0; mu < 4; ++mu)
        for (int c = 0; c < 3 * NR; ++c)
            for (int64_t s = 0; s < S; ++s) {
                const int64_t k = Lay::slot(mu, c, S, s);
                EXPECT(k >= 0 && k < n && !seen[k], "layout slot %lld reused or outside\n", (long long)k);
                if (k >= 0 && k < n) seen[k] = 1;
                if (Lay::kPaired && c < 8) {
                    const int64_t e = Lay::slot(mu, c & ~1, S, s);
                    EXPECT(e % 2 == 0 && Lay::slot(mu, c | 1, S, s) == e + 1, "FP32 pair not one 16-byte entry\n");
                }
            }
}

int main() {
    int n = 0;
    for (int64_t S : {256, 512, 4096}) {
        check_layout<double, 3>(S);
        check_layout<float, 3>(S);
        check_layout<float, 2>(S);
    }
    const int xs[] = {2, 3, 4, 8, 16, 24, 32, 48}, ys[] = {2, 4, 5, 8, 12}, zs[] = {2, 3, 4, 8}, ts[] = {2, 4, 6, 8, 16};
    for (int lx : xs)
        for (int ly : ys)
            for (int lz : zs)
                for (int lt : ts) {
                    const int32_t L[4] = {lx, ly, lz, lt};
                    check_lattice(L);
                    ++n;
                }
    const int32_t big[][4] = {{32, 32, 32, 64}, {16, 16, 16, 32}, {24, 24, 24, 48}, {20, 20, 20, 40}, {12, 12, 12, 24}};
    for (auto &L : big) {
        check_lattice(L);
        ++n;
    }
    for (int nb = 1; nb <= 4096; ++nb) {
        std::vector<int> img(nb);
        for (int b = 0; b < nb; ++b) img[b] = xcd_tile(b, nb);
        EXPECT(bijection(nb, img), "xcd_tile not a bijection for %d blocks\n", nb);
    }
    if (!fails) std::printf("ok %d lattices\n", n);
    return fails != 0;
}
