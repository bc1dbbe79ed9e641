// CPU test of the autotuner's JSON file (zb_tunecache.h): what the writer emits reads back
// the same, keys in another order and other whitespace read the same, and every malformed
// or out-of-range file is refused with the table untouched.
#include <stdio.h>

#include <random>
#include <string>
#include <vector>

#include "zb_tunecache.h"

using zbh::TuneEntry;

static int fails = 0;
#define CHECK(c)                                               \
    do {                                                       \
        if (!(c)) {                                            \
            printf("check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                           \
        }                                                      \
    } while (0)

static bool same(const std::vector<TuneEntry> &a, const std::vector<TuneEntry> &b)
{
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
        if (a[i].nv != b[i].nv || a[i].nr != b[i].nr || a[i].prec != b[i].prec ||
            a[i].lanes != b[i].lanes || a[i].auto_lanes != b[i].auto_lanes || a[i].auto_lu != b[i].auto_lu)
            return false;
    return true;
}

static bool parse(const std::string &t, std::vector<TuneEntry> &es, std::string &arch, int &rt)
{
    std::string err;
    return zbh::tune_parse(t, 64, 4096, arch, rt, es, err);
}

int main()
{
    // round trip, with random tables
    std::mt19937 g(3);
    for (int it = 0; it < 200; ++it) {
        std::vector<TuneEntry> es;
        const int n = g() % 9;
        for (int i = 0; i < n; ++i)
            es.push_back({1 + (int)(g() % 64), (int)(g() % 4097), (int)(g() % 2), 1 << (g() % 7),
                          1 << (g() % 7), (int)(g() % 2)});
        const std::string t = zbh::tune_json("gfx950:sramecc+:xnack-", 70226015, es);
        std::vector<TuneEntry> back;
        std::string arch;
        int rt = 0;
        CHECK(parse(t, back, arch, rt));
        CHECK(same(es, back));
        CHECK(arch == "gfx950:sramecc+:xnack-");
        CHECK(rt == 70226015);
    }
    printf("round trip ok\n");

    // the same content written by hand: keys reordered, other whitespace, escapes in a string
    {
        const std::string t =
            "\r\n{ \"entries\":[ {\"auto_lu\":1,\"auto_lanes\":64,\"lanes\":64,\"precision\":1,"
            "\"nr\":150,\"nv\":48}\t],\"hip_runtime\" : 7,\"arch\":\"gfx\\/950\",\"format\":"
            "\"zoneburn-tune-1\"}  ";
        std::vector<TuneEntry> es;
        std::string arch;
        int rt = 0;
        CHECK(parse(t, es, arch, rt));
        CHECK(es.size() == 1 && es[0].nv == 48 && es[0].nr == 150 && es[0].prec == 1 &&
              es[0].lanes == 64 && es[0].auto_lanes == 64 && es[0].auto_lu == 1);
        CHECK(arch == "gfx/950" && rt == 7);
    }
    printf("reordered ok\n");

    // the writer drops characters that would break the string
    {
        const std::string t = zbh::tune_json("gfx\"9\\50\n", 1, {});
        std::vector<TuneEntry> es;
        std::string arch;
        int rt = 0;
        CHECK(parse(t, es, arch, rt));
        CHECK(arch == "gfx950" && es.empty());
    }

    // refused: each case leaves the output table as it was
    const std::string good = zbh::tune_json("gfx950", 5, {{14, 30, 1, 16, 16, 0}});
    const char *bad[] = {
        "",
        "[]",
        "{}",
        "null",
        "{\"format\": \"zoneburn-tune-2\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": []}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": 950, \"hip_runtime\": 5, \"entries\": []}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": -1, \"entries\": []}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5.5, \"entries\": []}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": {}}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": [1]}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": "
        "[{\"nv\": 14, \"nr\": 30, \"precision\": 1, \"lanes\": 16, \"auto_lanes\": 16}]}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": "
        "[{\"nv\": 14, \"nr\": 30, \"precision\": 1, \"lanes\": 12, \"auto_lanes\": 16, \"auto_lu\": 0}]}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": "
        "[{\"nv\": 65, \"nr\": 30, \"precision\": 1, \"lanes\": 16, \"auto_lanes\": 16, \"auto_lu\": 0}]}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": "
        "[{\"nv\": 14, \"nr\": 4097, \"precision\": 1, \"lanes\": 16, \"auto_lanes\": 16, \"auto_lu\": 0}]}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": "
        "[{\"nv\": 14, \"nr\": 30, \"precision\": 2, \"lanes\": 16, \"auto_lanes\": 16, \"auto_lu\": 0}]}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": "
        "[{\"nv\": 14, \"nr\": 30, \"precision\": 1, \"lanes\": 16, \"auto_lanes\": 16, \"auto_lu\": 3}]}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": "
        "[{\"nv\": 14, \"nr\": 30, \"precision\": 1, \"lanes\": 16, \"auto_lanes\": 16, \"auto_lu\": 0, "
        "\"extra\": 1}]}",
        "{\"format\": \"zoneburn-tune-1\", \"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", "
        "\"hip_runtime\": 5, \"entries\": []}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 99999999999999999999, "
        "\"entries\": []}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx\\u0039\", \"hip_runtime\": 5, \"entries\": []}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": []} x",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": [],}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": [[[[[[[[[[]]]]]]]]]]}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\" \"hip_runtime\": 5, \"entries\": []}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": 5, \"entries\": [",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx9\n50\", \"hip_runtime\": 5, \"entries\": []}",
        "{\"format\": \"zoneburn-tune-1\", \"arch\": \"gfx950\", \"hip_runtime\": -, \"entries\": []}",
    };
    for (const char *b : bad) {
        std::vector<TuneEntry> es = {{3, 3, 0, 4, 4, 0}};
        std::string arch = "keep", err;
        int rt = 42;
        const bool ok = zbh::tune_parse(b, 64, 4096, arch, rt, es, err);
        CHECK(!ok);
        CHECK(!err.empty());
        CHECK(es.size() == 1 && es[0].nv == 3 && arch == "keep" && rt == 42);
        if (ok) printf("accepted: %s\n", b);
    }
    // every prefix of a good file that stops before its closing brace is refused as well
    CHECK(good.substr(good.size() - 3) == "]}\n");
    for (size_t n = 0; n + 2 < good.size(); ++n) {
        std::vector<TuneEntry> es;
        std::string arch, err;
        int rt = 0;
        CHECK(!zbh::tune_parse(good.substr(0, n), 64, 4096, arch, rt, es, err));
    }
    // random byte flips never crash the reader (the sanitizers watch)
    for (int it = 0; it < 20000; ++it) {
        std::string t = good;
        const int k = 1 + g() % 4;
        for (int j = 0; j < k; ++j) t[g() % t.size()] = (char)(g() % 256);
        std::vector<TuneEntry> es;
        std::string arch, err;
        int rt = 0;
        if (zbh::tune_parse(t, 64, 4096, arch, rt, es, err))
            for (auto &e : es) CHECK(e.nv >= 1 && e.nv <= 64 && e.nr >= 0 && e.nr <= 4096);
    }
    printf("refusals ok\n");
    if (fails) {
        printf("%d checks failed\n", fails);
        return 1;
    }
    printf("tunecache ok\n");
    return 0;
}
