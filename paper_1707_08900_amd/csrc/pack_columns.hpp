// Packed deal of the tile columns of a batched ensemble over the workgroups of
// the persistent launch (host code; the schedule FD6_BATCH_PACKED).  Plain
// C++17 with no HIP dependency, so the host tests compile it on their own.
#pragma once

#include <algorithm>
#include <functional>
#include <queue>
#include <utility>
#include <vector>

namespace fd6 {

// cols: whole tile columns (Item has int members box, x0, y0, zb, ze; here
// zb = 0 and ze = nz), in (box, y, x) order.  A piece of n planes costs
// n + refill plane steps (the pipeline refill of a work item).
//
// The columns are taken longest first, in the given order among equal lengths,
// and each goes to the least-loaded of the G workgroups (the lowest index
// among equals): the first G columns are neighbouring tiles swept at the same
// time.  A column that would take its workgroup past a target cost is cut
// where the workgroup reaches it, if both parts keep min_chunk planes, and its
// rest is queued again by length.  A cut workgroup holds exactly the target
// and is never cut again, so at most G columns are split.  Targets from the
// mean cost to the mean plus the longest column (where nothing is cut any
// more) are tried, and the deal with the smallest largest load, then the
// fewest pieces, is kept; the scan is skipped when the deal without cuts is
// already within 0.5% of the mean.
//
// Fills flat with the items of workgroups 0 .. G-1 in turn, each list in the
// order dealt, and first[L] with the offset of workgroup L's list (first[G] =
// flat->size()).
template <typename Item>
void pack_columns(const std::vector<Item>& cols, int G, int refill, int min_chunk,
                  std::vector<Item>* flat, std::vector<int>* first) {
    long long total = 0, longest = 0;
    for (const Item& c : cols) {
        const long long k = c.ze - c.zb + refill;
        total += k;
        longest = std::max(longest, k);
    }
    struct Piece {
        int len;
        long long seq;  // queue order among equal lengths
        int col, zb;
    };
    auto after = [](const Piece& a, const Piece& c) {
        return a.len != c.len ? a.len < c.len : a.seq > c.seq;
    };
    using Load = std::pair<long long, int>;  // (cost so far, workgroup)
    // Deals every column for one target; returns (largest load, pieces).
    auto deal = [&](long long target, std::vector<std::vector<Item>>* lists) {
        std::priority_queue<Piece, std::vector<Piece>, decltype(after)> q(after);
        for (size_t k = 0; k < cols.size(); ++k)
            q.push(Piece{cols[k].ze - cols[k].zb, (long long)k, (int)k, cols[k].zb});
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> wg;
        for (int j = 0; j < G; ++j) wg.push(Load{0, j});
        long long seq = (long long)cols.size(), largest = 0, npieces = 0;
        while (!q.empty()) {
            const Piece p = q.top();
            q.pop();
            Load l = wg.top();
            wg.pop();
            int take = p.len;
            const long long fit = target - l.first - refill;
            if (l.first + p.len + refill > target && fit >= min_chunk && p.len - fit >= min_chunk) {
                take = (int)fit;
                q.push(Piece{p.len - take, seq++, p.col, p.zb + take});
            }
            if (lists) {
                Item it = cols[p.col];
                it.zb = p.zb;
                it.ze = p.zb + take;
                (*lists)[l.second].push_back(it);
            }
            l.first += take + refill;
            largest = std::max(largest, l.first);
            ++npieces;
            wg.push(l);
        }
        return std::make_pair(largest, npieces);
    };
    // The deal without cuts (target lo + longest) first: when its largest load
    // is within 0.5% of the mean (many columns per workgroup), cuts cannot gain
    // more and the scan is skipped; otherwise targets lo, lo + stride, ...
    const long long lo = (total + G - 1) / G, hi = lo + longest;
    const long long stride = std::max<long long>(1, longest / 64);
    long long best_target = hi;
    std::pair<long long, long long> best = deal(hi, nullptr);
    if (best.first * 200 > lo * 201)
        for (long long t = lo; t < hi; t = std::min(t + stride, hi)) {
            const auto m = deal(t, nullptr);
            if (m < best) best = m, best_target = t;
        }
    std::vector<std::vector<Item>> lists(G);
    deal(best_target, &lists);
    flat->clear();
    first->assign(G + 1, 0);
    for (int L = 0; L < G; ++L) {
        (*first)[L] = (int)flat->size();
        flat->insert(flat->end(), lists[L].begin(), lists[L].end());
    }
    (*first)[G] = (int)flat->size();
}

}  // namespace fd6
