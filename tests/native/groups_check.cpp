// Host check of the batch engine's packing of bands into workgroup items
// (fhp_groups.h): every band of every member is in exactly one item; an item
// holds bands of one (wd, T) class that fit its workgroup; every wave holds
// bands of a single member; the lane -> band mapping that the kernel derives
// from a wave's descriptor gives each band wd lanes inside the workgroup; and
// the queue runs items by decreasing band height.  Prints OK on success.
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <random>
#include <utility>
#include <vector>

#include "fhp_groups.h"

using namespace fhp;

static int fails = 0;
#define CHECK(c, ...)                              \
    do {                                           \
        if (!(c)) {                                \
            if (fails++ < 10) {                    \
                printf("FAIL %s: ", #c);           \
                printf(__VA_ARGS__);               \
                printf("\n");                      \
            }                                      \
        }                                          \
    } while (0)

static void check_case(const std::vector<MemberBands>& mem, uint32_t nt, int id) {
    std::vector<GroupDesc> groups;
    std::vector<WaveDesc> waves;
    std::vector<uint32_t> lanes;
    pack_waves(mem, nt, groups, waves, lanes);
    CHECK(groups.size() == lanes.size(), "case %d lanes table", id);
    // lanes per group before ordering, keyed by first wave (unique per group)
    std::map<uint32_t, uint32_t> used_of;
    for (size_t g = 0; g < groups.size(); g++) used_of[groups[g].first_wave] = lanes[g];
    order_groups(groups, lanes);

    uint64_t total_bands = 0, total_lanes = 0;
    std::map<uint32_t, const MemberBands*> by_m;
    for (const MemberBands& mb : mem) {
        by_m[mb.m] = &mb;
        total_bands += mb.nbands;
        total_lanes += (uint64_t)mb.nbands * mb.wd;
    }
    CHECK(waves.size() <= max_waves(total_bands), "case %d: %zu waves > bound", id, waves.size());
    std::map<std::pair<uint32_t, uint32_t>, int> seen;  // (member, band) -> count
    uint32_t prev_T = ~0u;
    for (size_t g = 0; g < groups.size(); g++) {
        const GroupDesc& G = groups[g];
        CHECK(G.nwaves >= 1 && G.nwaves * 64 <= nt, "case %d group %zu nwaves %u", id, g, G.nwaves);
        CHECK(G.first_wave + G.nwaves <= waves.size(), "case %d group %zu range", id, g);
        // the kernel's lane mapping, lane by lane
        std::map<std::pair<uint32_t, uint32_t>, uint32_t> lanes_of_band;
        uint32_t used = 0;
        for (uint32_t lane = 0; lane < nt; lane++) {
            const uint32_t wave = lane / 64;
            if (wave >= G.nwaves) continue;
            const WaveDesc& D = waves[G.first_wave + wave];
            const MemberBands* mb = by_m.count(D.m) ? by_m[D.m] : nullptr;
            CHECK(mb != nullptr, "case %d unknown member %u", id, D.m);
            if (!mb) continue;
            CHECK(mb->wd == G.wd && mb->T == G.T, "case %d group %zu mixes classes", id, g);
            CHECK(D.rel0 % 64 == 0, "case %d rel0 %u", id, D.rel0);
            const uint32_t rel = D.rel0 + (lane & 63);
            const uint32_t j = rel / G.wd, w = rel - j * G.wd;
            if (j >= D.count) continue;
            const uint32_t b = D.band0 + j;
            CHECK(b < mb->nbands, "case %d band %u of %u", id, b, mb->nbands);
            const uint32_t first = lane - w;
            CHECK(first + G.wd <= nt, "case %d band lanes leave the workgroup", id);
            // every lane of the band is in a wave of the same run
            for (uint32_t q = first; q < first + G.wd && q < nt; q++) {
                const uint32_t wq = q / 64;
                CHECK(wq < G.nwaves, "case %d band lane %u in an idle wave", id, q);
                if (wq >= G.nwaves) continue;
                const WaveDesc& E = waves[G.first_wave + wq];
                CHECK(E.m == D.m && E.band0 == D.band0 && E.count == D.count &&
                          E.rel0 - D.rel0 == 64 * (wq - wave),
                      "case %d band straddles runs", id);
            }
            lanes_of_band[{D.m, b}]++;
            used++;
        }
        for (auto& kv : lanes_of_band) {
            CHECK(kv.second == G.wd, "case %d member %u band %u has %u lanes", id, kv.first.first,
                  kv.first.second, kv.second);
            seen[kv.first]++;
        }
        CHECK(used_of.count(G.first_wave) && used_of[G.first_wave] == used,
              "case %d group %zu lane count", id, g);
        CHECK(G.T <= prev_T, "case %d queue order at %zu", id, g);
        prev_T = G.T;
        total_lanes -= used;
    }
    CHECK(total_lanes == 0, "case %d lanes left over", id);
    for (const MemberBands& mb : mem)
        for (uint32_t b = 0; b < mb.nbands; b++) {
            const int k = seen[std::make_pair(mb.m, b)];
            CHECK(k == 1, "case %d member %u band %u covered %d times", id, mb.m, b, k);
        }
}

int main() {
    std::mt19937_64 rng(12345);
    int id = 0;
    // small lattices packed many to a wave, one member per wave
    {
        std::vector<MemberBands> mem;
        for (uint32_t i = 0; i < 10; i++) mem.push_back({i, 2, 32, 4});  // 8 lanes each
        check_case(mem, 256, id++);
        std::vector<GroupDesc> g;
        std::vector<WaveDesc> w;
        std::vector<uint32_t> l;
        pack_waves(mem, 256, g, w, l);
        CHECK(g.size() == 3 && w.size() == 10, "10 members of 8 lanes: %zu groups %zu waves",
              g.size(), w.size());  // one wave each, four waves per workgroup
    }
    // a band wider than a wave spans waves of one run
    {
        std::vector<MemberBands> mem = {{0, 100, 16, 5}, {1, 100, 16, 3}};
        check_case(mem, 256, id++);
    }
    // random mixes of widths, band heights and band counts, members listed
    // class by class as the engine does
    for (int c = 0; c < 300; c++) {
        const int n = 1 + (int)(rng() % 120);
        std::vector<MemberBands> mem;
        uint32_t max_wd = 1;
        for (int i = 0; i < n; i++) {
            const uint32_t wd = 1u + (uint32_t)(rng() % ((c % 3 == 0) ? 512 : 40));
            const uint32_t T = 2u * (1u + (uint32_t)(rng() % 4));
            mem.push_back({(uint32_t)(1000 + i), wd, T, 1u + (uint32_t)(rng() % 40)});
            max_wd = std::max(max_wd, wd);
        }
        std::stable_sort(mem.begin(), mem.end(), [](const MemberBands& a, const MemberBands& b) {
            if (a.wd != b.wd) return a.wd > b.wd;
            return a.T > b.T;
        });
        uint32_t nt = 64u << (rng() % 4);
        if (nt < (max_wd + 63) / 64 * 64) nt = (max_wd + 63) / 64 * 64;
        check_case(mem, nt, id++);
    }
    if (fails) {
        printf("%d failures\n", fails);
        return 1;
    }
    printf("OK %d cases\n", id);
    return 0;
}
