// fhp_groups.h -- host-side packing of lattice bands into workgroup items for
// the batch kernel (plain C++: also built on the host alone to be checked).
//
// A band is T consecutive rows of one lattice over its full width (wd 64-node
// words, one lane per word).  A work item is one workgroup of nt lanes; all
// its bands share wd and T, so every wave of the item sweeps the same rows in
// lockstep.  Each wave holds bands of a single lattice (a run of consecutive
// bands that starts on a wave boundary, possibly spanning several waves), so
// that every per-lattice value -- buffers, keys, time, walls, forcing -- is
// uniform across the wave and lives in scalar registers.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace fhp {

// One item: waves [first_wave, first_wave + nwaves) of the wave table; the
// workgroup's remaining waves idle.
struct GroupDesc {
    uint32_t wd, T;
    uint32_t first_wave, nwaves;
};

// One wave of an item: lanes of bands band0 .. band0 + count - 1 of member m,
// laid side by side from the run's first lane; rel0 = lanes of the run that
// precede this wave's lane 0 (a multiple of 64).
struct WaveDesc {
    uint32_t m, band0, count, rel0;
};

// A member's bands, in the order the members are packed.
struct MemberBands {
    uint32_t m, wd, T, nbands;
};

// Upper bound on the wave-table entries for `bands` bands of at most 512
// words: a run of c bands of width wd spans ceil(c wd / 64) <= c wd / 64 + 1
// waves, and there are at most `bands` runs.
inline uint64_t max_waves(uint64_t bands) { return bands * 9; }

// Packs the bands of `mem` (listed class by class, a class being equal
// (wd, T)) into items of nt lanes.  Appends to groups / waves and returns the
// lanes holding a band in each group via `lanes` (same length as groups).
inline void pack_waves(const std::vector<MemberBands>& mem, uint32_t nt,
                       std::vector<GroupDesc>& groups, std::vector<WaveDesc>& waves,
                       std::vector<uint32_t>& lanes) {
    groups.clear();
    waves.clear();
    lanes.clear();
    bool open = false;
    GroupDesc g{};
    uint32_t pos = 0, used = 0;  // next free lane (a wave boundary), lanes holding bands
    auto close = [&]() {
        if (open && g.nwaves) {
            groups.push_back(g);
            lanes.push_back(used);
        }
        open = false;
    };
    for (const MemberBands& mb : mem) {
        if (open && (g.wd != mb.wd || g.T != mb.T)) close();
        uint32_t b = 0;
        while (b < mb.nbands) {
            if (!open) {
                g = GroupDesc{mb.wd, mb.T, (uint32_t)waves.size(), 0};
                pos = used = 0;
                open = true;
            }
            const uint32_t fit = (nt - pos) / mb.wd;
            if (fit == 0) {
                close();
                continue;
            }
            const uint32_t cnt = std::min(mb.nbands - b, fit);
            const uint32_t nw = (cnt * mb.wd + 63) / 64;
            for (uint32_t k = 0; k < nw; k++) waves.push_back({mb.m, b, cnt, 64 * k});
            g.nwaves += nw;
            pos += 64 * nw;
            used += cnt * mb.wd;
            b += cnt;
            if (pos >= nt) close();
        }
    }
    close();
}

// Queue order: most rows first (stable).  An item's time follows its band
// height, not its lane count (its waves run side by side); among equal
// heights the packing order is kept, so a member's bands stay together in
// the queue (the 512-lattice ensemble measured 1% faster than with items
// ordered by lanes x rows).
inline void order_groups(std::vector<GroupDesc>& groups, const std::vector<uint32_t>& lanes) {
    (void)lanes;
    std::vector<uint32_t> idx(groups.size());
    for (uint32_t k = 0; k < idx.size(); k++) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](uint32_t x, uint32_t y) { return groups[x].T > groups[y].T; });
    std::vector<GroupDesc> out(groups.size());
    for (uint32_t k = 0; k < idx.size(); k++) out[k] = groups[idx[k]];
    groups.swap(out);
}

}  // namespace fhp
