// Host check of the batch engine's packing of bands into workgroup items
// (fhp_groups.h): every band is in exactly one item, an item holds bands of
// one class that fit its workgroup, the last round of a pass is split into
// one-wave pieces, and the queue runs full items first, then the rest by
// decreasing work.  Prints OK on success.
#include <stdio.h>
#include <stdlib.h>

#include <random>
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

struct Mem {
    uint32_t wd, H, T;
    uint64_t ps;
};

static void check_case(const std::vector<Mem>& mem, uint32_t nt, uint32_t grid, int id) {
    // list bands class by class, as the engine does after sorting its members
    std::vector<uint32_t> order(mem.size());
    for (uint32_t i = 0; i < mem.size(); i++) order[i] = i;
    std::sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        const Mem &a = mem[x], &b = mem[y];
        if (a.wd != b.wd) return a.wd > b.wd;
        if (a.H != b.H) return a.H > b.H;
        if (a.T != b.T) return a.T > b.T;
        if (a.ps != b.ps) return a.ps > b.ps;
        return x < y;
    });
    std::vector<BandSeg> segs;
    for (uint32_t i : order)
        for (uint32_t b = 0; b < mem[i].H / mem[i].T; b++)
            segs.push_back({mem[i].wd, mem[i].T, mem[i].H, i, b, mem[i].ps});
    std::vector<GroupDesc> groups;
    std::vector<uint32_t> sm(segs.size()), sb(segs.size());
    pack_groups(segs, nt, groups, sm.data(), sb.data());
    const size_t G0 = groups.size();
    size_t unsplittable = 0;  // groups of one wave or less cannot be split
    for (const GroupDesc& g : groups) unsplittable += g.nseg <= (g.wd >= 64 ? 1u : 64u / g.wd);
    split_last_round(groups, nt, grid);
    order_groups(groups, nt);

    std::vector<int> seen(segs.size(), 0);
    for (size_t k = 0; k < segs.size(); k++) {
        CHECK(sm[k] == segs[k].m && sb[k] == segs[k].band, "case %d seg %zu tables", id, k);
    }
    for (size_t j = 0; j < groups.size(); j++) {
        const GroupDesc& g = groups[j];
        CHECK(g.nseg >= 1 && g.nseg * g.wd <= nt, "case %d group %zu nseg %u wd %u nt %u", id, j,
              g.nseg, g.wd, nt);
        CHECK(g.first + g.nseg <= segs.size(), "case %d group %zu range", id, j);
        for (uint32_t k = g.first; k < g.first + g.nseg && k < segs.size(); k++) {
            seen[k]++;
            const BandSeg& s = segs[k];
            CHECK(s.wd == g.wd && s.T == g.T && s.H == g.H && s.ps == g.ps,
                  "case %d group %zu mixes classes", id, j);
        }
    }
    for (size_t k = 0; k < segs.size(); k++)
        CHECK(seen[k] == 1, "case %d seg %zu covered %d times", id, k, seen[k]);
    // queue order: full groups, then part-filled ones by decreasing work
    size_t nfull = 0;
    while (nfull < groups.size() && groups[nfull].nseg == nt / groups[nfull].wd) nfull++;
    for (size_t j = nfull; j < groups.size(); j++) {
        CHECK(groups[j].nseg < nt / groups[j].wd, "case %d full group %zu after a part-filled one",
              id, j);
        if (j > nfull)
            CHECK(group_work(groups[j - 1]) >= group_work(groups[j]), "case %d order at %zu", id, j);
    }
    // the last round: with rem = G0 mod grid groups in it, the rem largest
    // are split, so at most G0 - rem + unsplittable full-size groups remain
    if (grid && G0 > grid && G0 % grid && nt > 64) {
        const size_t rem = G0 % grid;
        CHECK(nfull <= G0 - rem + unsplittable, "case %d: %zu full groups of %zu, last round %zu",
              id, nfull, G0, rem);
        CHECK(groups.size() >= G0, "case %d lost groups", id);
    } else {
        CHECK(groups.size() == G0, "case %d split without a last round", id);
    }
}

int main() {
    std::mt19937_64 rng(12345);
    int id = 0;
    // one class, every group full except the last: the split leaves exactly
    // whole rounds of full groups
    {
        std::vector<Mem> mem;
        for (int i = 0; i < 100; i++) mem.push_back({8, 256, 32, 8 * 256});
        const uint32_t nt = 256, grid = 64;  // 800 bands, 32 per group -> 25 groups
        check_case(mem, nt, grid, id++);
        check_case(mem, nt, 16, id++);       // 25 = 16 + 9
        std::vector<BandSeg> segs;
        for (uint32_t i = 0; i < mem.size(); i++)
            for (uint32_t b = 0; b < 8; b++) segs.push_back({8, 32, 256, i, b, 8 * 256});
        std::vector<GroupDesc> g;
        std::vector<uint32_t> sm(segs.size()), sb(segs.size());
        pack_groups(segs, nt, g, sm.data(), sb.data());
        CHECK(g.size() == 25, "groups %zu", g.size());
        split_last_round(g, nt, 16);
        order_groups(g, nt);
        size_t full = 0;
        for (auto& x : g) full += x.nseg == 32;
        CHECK(full == 16, "full groups after split %zu", full);
        CHECK(g.size() == 16 + 9 * 4, "pieces %zu", g.size());  // 32 bands -> 4 one-wave pieces
    }
    // random mixes of widths, heights and band heights
    for (int c = 0; c < 300; c++) {
        const int n = 1 + (int)(rng() % 200);
        std::vector<Mem> mem;
        uint32_t max_wd = 1;
        for (int i = 0; i < n; i++) {
            const uint32_t wd = 1u + (uint32_t)(rng() % ((c % 3 == 0) ? 512 : 40));
            const uint32_t T = 2u * (1u + (uint32_t)(rng() % 32));
            const uint32_t H = T * (1u + (uint32_t)(rng() % 40));
            mem.push_back({wd, H, T, (uint64_t)wd * H + (rng() % 2) * 32});
            max_wd = std::max(max_wd, wd);
        }
        uint32_t nt = 64u << (rng() % 4);
        if (nt < (max_wd + 63) / 64 * 64) nt = (max_wd + 63) / 64 * 64;
        const uint32_t grid = (uint32_t)(rng() % 3000);
        check_case(mem, nt, grid, id++);
    }
    if (fails) {
        printf("%d failures\n", fails);
        return 1;
    }
    printf("OK %d cases\n", id);
    return 0;
}
