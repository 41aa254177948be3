// Host check of the launch-table file reader and writer (tunecache.cpp):
//  * a written table reads back entry for entry;
//  * a missing file reads as "no such file", a table recorded on another
//    architecture as "other architecture" with no entries;
//  * malformed files (not JSON, trailing text, wrong types, unknown names,
//    non-integer or out-of-range numbers, truncated text) are refused with
//    a message, never read partially;
//  * unknown keys and extra whitespace are accepted.
// Prints "ok" and the number of cases checked.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_1105_2279_amd/csrc/qdpx_impl.hpp"

using namespace qdpx;

static int fails = 0, cases = 0;
#define EXPECT(cond, ...)                             \
    do {                                              \
        ++cases;                                      \
        if (!(cond)) {                                \
            if (fails < 20) std::printf(__VA_ARGS__); \
            ++fails;                                  \
        }                                             \
    } while (0)

static void put(const std::string &path, const std::string &text) {
    FILE *f = std::fopen(path.c_str(), "wb");
    std::fwrite(text.data(), 1, text.size(), f);
    std::fclose(f);
}

int main(int argc, char **argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    const std::string path = dir + "/table.json";
    std::string err;
    std::vector<TuneEntry> in, out;
    for (int op = 0; op < 6; ++op)
        for (int prec = 0; prec < 2; ++prec) {
            TuneEntry t;
            t.op = op;
            t.prec = prec;
            t.fmt = prec;  // LINK12 with F32
            t.L[0] = 8 + op;
            t.L[1] = 4;
            t.L[2] = 6 + prec;
            t.L[3] = 16;
            t.cfg.block = 256 << prec;
            t.cfg.nsite = 1 + op % 3;
            t.cfg.xcd = op % 3;
            t.cfg.tw = 1 << (op % 4);
            t.cfg.lds = (op + prec) % 3;
            in.push_back(t);
        }
    EXPECT(tune_table_write(path.c_str(), "gfx950:sramecc+:xnack-", in, err) == 0, "write failed: %s\n", err.c_str());
    EXPECT(tune_table_read(path.c_str(), "gfx950", out, err) == 0, "read failed: %s\n", err.c_str());
    EXPECT(out.size() == in.size(), "read %zu of %zu entries\n", out.size(), in.size());
    for (size_t i = 0; i < out.size() && i < in.size(); ++i) {
        const TuneEntry &a = in[i], &b = out[i];
        EXPECT(a.op == b.op && a.prec == b.prec && a.fmt == b.fmt && a.L[0] == b.L[0] && a.L[1] == b.L[1] &&
                   a.L[2] == b.L[2] && a.L[3] == b.L[3] && a.cfg.block == b.cfg.block && a.cfg.nsite == b.cfg.nsite &&
                   a.cfg.xcd == b.cfg.xcd && a.cfg.tw == b.cfg.tw && a.cfg.lds == b.cfg.lds,
               "entry %zu differs after the round trip\n", i);
    }
    EXPECT(tune_table_read(path.c_str(), "gfx942:sramecc+", out, err) == 2 && out.empty(),
           "another architecture was not reported\n");
    EXPECT(tune_table_read((dir + "/missing.json").c_str(), "gfx950", out, err) == 1, "missing file not reported\n");

    const std::string good =
        "{\"device\": \"gfx950\", \"x\": [1, {\"y\": null}, true, false, -2.5e3, \"a\\\"b\\u0041\"],\n"
        "  \"entries\": [ {\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", \"L\": [32, 32, 32, 64],\n"
        "                 \"launch\": [512, 1, 2, 1], \"note\": \"tuned\"} ] }\n";
    put(path, good);
    EXPECT(tune_table_read(path.c_str(), "gfx950", out, err) == 0 && out.size() == 1 && out[0].op == 2 &&
               out[0].prec == 1 && out[0].fmt == 1 && out[0].L[3] == 64 && out[0].cfg.block == 512 &&
               out[0].cfg.xcd == 2 && out[0].cfg.lds == -1,
           "a table with extra keys (and no LDS tile field) was not read: %s\n", err.c_str());
    put(path, "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", "
              "\"L\": [8, 8, 8, 8], \"launch\": [256, 1, 1, 1, 2]}]}");
    EXPECT(tune_table_read(path.c_str(), "gfx950", out, err) == 0 && out.size() == 1 && out[0].cfg.lds == 2,
           "the LDS tile field was not read: %s\n", err.c_str());

    const char *bad[] = {
        "",
        "not json",
        "{\"device\": \"gfx950\", \"entries\": []} trailing",
        "{\"device\": \"gfx950\"}",
        "{\"entries\": []}",
        "{\"device\": 950, \"entries\": []}",
        "{\"device\": \"gfx950\", \"entries\": {}}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"XYZ\", \"prec\": \"F32\", \"fmt\": \"LINK12\", "
        "\"L\": [8, 8, 8, 8], \"launch\": [256, 1, 1, 1]}]}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F16\", \"fmt\": \"LINK12\", "
        "\"L\": [8, 8, 8, 8], \"launch\": [256, 1, 1, 1]}]}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", "
        "\"L\": [8, 8, 8], \"launch\": [256, 1, 1, 1]}]}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", "
        "\"L\": [8, 8, 8, 8.5], \"launch\": [256, 1, 1, 1]}]}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", "
        "\"L\": [8, 8, 8, 1e300], \"launch\": [256, 1, 1, 1]}]}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", "
        "\"L\": [8, 8, 8, 8], \"launch\": [\"256\", 1, 1, 1]}]}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", "
        "\"L\": [8, 8, 8, 8], \"launch\": [256, 1, 1, 1]}",
        "{\"device\": \"gfx950\", \"entries\": [1, 2]}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", "
        "\"L\": [8, 8, 8, 8], \"launch\": [256, 1, 1, 1, 2, 0]}]}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", "
        "\"L\": [8, 8, 8, 8], \"launch\": [256, 1, 1]}]}",
        "{\"device\": \"gfx950\", \"entries\": [{\"op\": \"APE\",}]}",
        "{\"device\": \"gfx\\q950\", \"entries\": []}",
        "[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]"
        "]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]",
    };
    for (const char *b : bad) {
        put(path, b);
        err.clear();
        const int r = tune_table_read(path.c_str(), "gfx950", out, err);
        EXPECT(r == -1 && out.empty() && !err.empty(), "malformed table accepted (r = %d): %s\n", r, b);
    }
    std::remove(path.c_str());
    if (fails) {
        std::printf("%d of %d checks failed\n", fails, cases);
        return 1;
    }
    std::printf("ok %d checks\n", cases);
    return 0;
}
