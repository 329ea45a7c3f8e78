// fhp_groups.h -- host-side packing of lattice bands into workgroup items for
// the batch kernel (plain C++: also built on the host alone to be checked).
//
// A band is T consecutive rows of one lattice over its full width (wd 64-node
// words).  Bands of lattices with the same width, height, band height and
// plane stride share a workgroup of nt threads, nt / wd of them side by side;
// the persistent grid takes the resulting items from one queue.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace fhp {

struct GroupDesc {
    uint32_t first, nseg, wd, T, H, pad;
    uint64_t ps;  // plane stride in words
};

struct BandSeg {
    uint32_t wd, T, H, m, band;
    uint64_t ps;
};

inline bool same_class(const BandSeg& a, const BandSeg& b) {
    return a.wd == b.wd && a.T == b.T && a.H == b.H && a.ps == b.ps;
}

inline uint64_t group_work(const GroupDesc& g) { return (uint64_t)g.nseg * g.wd * g.T; }

// Packs segs (listed class by class) into groups of at most nt / wd bands;
// sm / sb receive each segment's member and band in the same order.
inline void pack_groups(const std::vector<BandSeg>& segs, uint32_t nt, std::vector<GroupDesc>& groups,
                        uint32_t* sm, uint32_t* sb) {
    groups.clear();
    for (size_t k = 0; k < segs.size();) {
        GroupDesc g{};
        g.first = (uint32_t)k;
        g.wd = segs[k].wd;
        g.T = segs[k].T;
        g.H = segs[k].H;
        g.ps = segs[k].ps;
        const uint32_t cap = nt / g.wd;
        const size_t k0 = k;
        while (k < segs.size() && g.nseg < cap && same_class(segs[k], segs[k0])) {
            sm[k] = segs[k].m;
            sb[k] = segs[k].band;
            g.nseg++;
            k++;
        }
        groups.push_back(g);
    }
}

// When a pass has a few full rounds of items on the persistent grid plus a
// part-filled last one, most of the grid idles while that last round runs.
// The groups that would make it up (the largest, which run first) are split
// into one-wave pieces, which run last and spread that work over the whole
// grid.  Segments stay consecutive, so only the group table changes.
inline void split_last_round(std::vector<GroupDesc>& groups, uint32_t nt, uint32_t grid) {
    const size_t G = groups.size();
    if (!grid || G <= grid || G % grid == 0 || nt <= 64) return;
    const size_t rem = G % grid;
    std::vector<size_t> idx(G);
    for (size_t k = 0; k < G; k++) idx[k] = k;
    std::nth_element(idx.begin(), idx.begin() + (rem - 1), idx.end(),
                     [&](size_t x, size_t y) { return group_work(groups[x]) > group_work(groups[y]); });
    std::vector<GroupDesc> pieces;
    for (size_t r = 0; r < rem; r++) {
        GroupDesc& g = groups[idx[r]];
        const uint32_t per = g.wd >= 64 ? 1u : 64u / g.wd;  // bands in one wave's worth
        if (g.nseg <= per) continue;
        for (uint32_t k = per; k < g.nseg; k += per) {
            GroupDesc q = g;
            q.first = g.first + k;
            q.nseg = g.nseg - k < per ? g.nseg - k : per;
            pieces.push_back(q);
        }
        g.nseg = per;
    }
    groups.insert(groups.end(), pieces.begin(), pieces.end());
}

// Queue order, largest work first: full groups in their class order ahead of
// the few part-filled ones, which are sorted among themselves.
inline void order_groups(std::vector<GroupDesc>& groups, uint32_t nt) {
    auto part = std::stable_partition(groups.begin(), groups.end(),
                                      [&](const GroupDesc& g) { return g.nseg == nt / g.wd; });
    std::stable_sort(part, groups.end(), [](const GroupDesc& x, const GroupDesc& y) {
        return group_work(x) > group_work(y);
    });
}

}  // namespace fhp
