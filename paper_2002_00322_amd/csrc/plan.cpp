// Host planning of the grouped J/K build (see plan.h).
#include "plan.h"

#include <algorithm>
#include <cstddef>
#include <numeric>

namespace esmf {

namespace {

// Recursive coordinate bisection of idx[lo, hi) into tiles of kTile slots.
void rcb(const double* centers, std::vector<int>& idx, size_t lo, size_t hi, std::vector<int32_t>& slot_fn) {
    const size_t cnt = hi - lo;
    if (cnt <= (size_t)kTile) {
        for (size_t t = 0; t < (size_t)kTile; ++t) slot_fn.push_back(t < cnt ? idx[lo + t] : -1);
        return;
    }
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (size_t t = lo; t < hi; ++t)
        for (int x = 0; x < 3; ++x) {
            mn[x] = std::min(mn[x], centers[3 * idx[t] + x]);
            mx[x] = std::max(mx[x], centers[3 * idx[t] + x]);
        }
    int ax = 0;
    for (int x = 1; x < 3; ++x)
        if (mx[x] - mn[x] > mx[ax] - mn[ax]) ax = x;
    std::stable_sort(idx.begin() + lo, idx.begin() + hi, [&](int a, int b) {
        const double ca = centers[3 * a + ax], cb = centers[3 * b + ax];
        if (ca != cb) return ca < cb;
        return a < b;
    });
    const size_t ntile = (cnt + kTile - 1) / kTile;
    const size_t left = (ntile / 2) * kTile;
    rcb(centers, idx, lo, lo + left, slot_fn);
    rcb(centers, idx, lo + left, hi, slot_fn);
}

// Spread bra rows (groups of items) over `xcd` queues, largest first onto the
// least loaded queue, and interleave the queues: item i of the result runs on
// XCD i % xcd (workgroups are dispatched round-robin over the XCDs).  When a
// queue runs dry its turn goes to the fullest one.
std::vector<WorkItem> interleave(const std::vector<std::vector<WorkItem>>& groups, int xcd) {
    std::vector<size_t> order(groups.size());
    std::iota(order.begin(), order.end(), 0);
    auto gsize = [&](size_t g) {
        int64_t n = 0;
        for (const WorkItem& it : groups[g]) n += it.e1 - it.e0;
        return n;
    };
    std::vector<int64_t> sizes(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) sizes[g] = gsize(g);
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return sizes[x] > sizes[y]; });
    std::vector<std::vector<WorkItem>> q(xcd);
    std::vector<int64_t> load(xcd, 0);
    for (size_t g : order) {
        const int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (const WorkItem& it : groups[g]) q[best].push_back(it);
        load[best] += sizes[g];
    }
    std::vector<WorkItem> items;
    std::vector<size_t> pos(xcd, 0);
    size_t remaining = 0;
    for (auto& x : q) remaining += x.size();
    items.reserve(remaining);
    while (remaining > 0) {
        for (int x = 0; x < xcd && remaining > 0; ++x) {
            int src = x;
            if (pos[src] >= q[src].size()) {
                src = 0;
                for (int y = 1; y < xcd; ++y)
                    if (q[y].size() - pos[y] > q[src].size() - pos[src]) src = y;
            }
            items.push_back(q[src][pos[src]++]);
            --remaining;
        }
    }
    return items;
}

// Slot numbering by target: new slot = start of its target's range + rank of
// the slot within its target in creation order.
void renumber(const std::vector<int64_t>& tgt, int64_t ntargets, std::vector<int64_t>& ptr,
              std::vector<int32_t>& newid) {
    ptr.assign((size_t)ntargets + 1, 0);
    for (int64_t t : tgt) ptr[(size_t)t + 1]++;
    for (size_t x = 0; x < (size_t)ntargets; ++x) ptr[x + 1] += ptr[x];
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    newid.resize(tgt.size());
    for (size_t x = 0; x < tgt.size(); ++x) newid[x] = (int32_t)fill[(size_t)tgt[x]]++;
}

}  // namespace

std::vector<int32_t> make_tile_plan(int n, const double* centers, const double* alpha) {
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (alpha[a] != alpha[b]) return alpha[a] < alpha[b];
        return a < b;
    });
    std::vector<int32_t> slot_fn;
    size_t g0 = 0;
    while (g0 < (size_t)n) {
        size_t g1 = g0;
        // one exponent class, extended by the following classes while it is
        // smaller than a tile
        while (g1 < (size_t)n) {
            size_t e = g1;
            while (e < (size_t)n && alpha[order[e]] == alpha[order[g1]]) ++e;
            g1 = e;
            if (g1 - g0 >= (size_t)kTile) break;
        }
        std::vector<int> grp(order.begin() + g0, order.begin() + g1);
        rcb(centers, grp, 0, grp.size(), slot_fn);
        g0 = g1;
    }
    return slot_fn;
}

void plan_blocks(const std::vector<double>& q, const std::vector<int32_t>& slot_fn, double tau, BlockList& bl) {
    const int ns = (int)slot_fn.size();
    const int nt = ns / kTile;
    bl.nslots = ns;
    bl.ntiles = nt;
    bl.slot_fn = slot_fn;
    bl.nbf = 0;
    for (int32_t f : slot_fn) bl.nbf += f >= 0;
    bl.blk_tiles.clear();
    bl.weight.clear();
    double qmax = 0.0;
    for (double v : q) qmax = std::max(qmax, v);
    // tile pairs (I >= J) whose largest factor can pass with some partner
    std::vector<int32_t> tpI, tpJ;
    std::vector<double> tpq;
    for (int I = 0; I < nt; ++I)
        for (int J = 0; J <= I; ++J) {
            double m = 0.0;
            for (int i = 0; i < kTile; ++i)
                for (int j = 0; j < kTile; ++j) m = std::max(m, q[(size_t)(I * kTile + i) * ns + (J * kTile + j)]);
            if (m * qmax > tau) {
                tpI.push_back(I);
                tpJ.push_back(J);
                tpq.push_back(m);
            }
        }
    for (size_t x = 0; x < tpI.size(); ++x)
        for (size_t y = 0; y <= x; ++y) {
            if (!(tpq[x] * tpq[y] > tau)) continue;
            bl.blk_tiles.push_back(tpI[x]);
            bl.blk_tiles.push_back(tpJ[x]);
            bl.blk_tiles.push_back(tpI[y]);
            bl.blk_tiles.push_back(tpJ[y]);
            double w = 1.0;
            if (tpI[x] == tpJ[x]) w *= 0.5;
            if (tpI[y] == tpJ[y]) w *= 0.5;
            if (x == y) w *= 0.5;
            bl.weight.push_back(w);
        }
}

int default_item_blocks(int kind, int64_t nblocks) {
    // entries per launch: two per block for two visits, one when fused
    const int64_t total = (kind == kPlanFused ? 1 : 2) * nblocks;
    const int64_t seg = total / (4 * 512);
    return (int)std::max<int64_t>(8, std::min<int64_t>(64, seg));
}

int plan_work(const BlockList& bl, int kind, int seg, int band, int xcd, WorkPlan& wp) {
    const std::vector<int32_t>& bt = bl.blk_tiles;
    const int64_t nb = bl.nblocks();
    const int T = bl.ntiles;
    seg = std::max(seg, 1);
    band = std::max(1, std::min(band, kMaxBand));
    xcd = std::max(xcd, 1);
    wp = WorkPlan();
    wp.kind = kind;
    wp.seg = seg;
    wp.band = kind == kPlanFused ? band : 0;
    std::vector<int32_t>& entries = wp.entries;
    entries.reserve((size_t)(kind == kPlanFused ? 1 : 2) * (size_t)nb);
    std::vector<std::vector<WorkItem>> groups;
    int64_t b0 = 0;
    while (b0 < nb) {
        int64_t b1 = b0;
        while (b1 < nb && bt[4 * b1] == bt[4 * b0] && bt[4 * b1 + 1] == bt[4 * b0 + 1]) ++b1;
        const int32_t I = bt[4 * b0], J = bt[4 * b0 + 1];
        groups.emplace_back();
        if (kind == kPlanTwoVisit) {
            // visit 0 walks the row in (K, L) order (the generation order),
            // visit 1 in (L, K) order; rows cut into items of seg blocks
            for (int visit = 0; visit < 2; ++visit) {
                std::vector<int32_t> row;
                for (int64_t b = b0; b < b1; ++b) row.push_back((int32_t)b);
                if (visit == 1)
                    std::stable_sort(row.begin(), row.end(), [&](int32_t x, int32_t y) {
                        if (bt[4 * x + 3] != bt[4 * y + 3]) return bt[4 * x + 3] < bt[4 * y + 3];
                        return bt[4 * x + 2] < bt[4 * y + 2];
                    });
                for (size_t r0 = 0; r0 < row.size(); r0 += (size_t)seg) {
                    const size_t r1 = std::min(row.size(), r0 + (size_t)seg);
                    WorkItem it{(int32_t)entries.size(), (int32_t)(entries.size() + (r1 - r0)), I, J, visit, 0, -1, 0};
                    for (size_t r = r0; r < r1; ++r) entries.push_back(row[r]);
                    groups.back().push_back(it);
                }
            }
        } else {
            // fused: the row's distinct L values in bands of `band`; a band's
            // blocks in (K, L) order, cut into items at K-run boundaries
            // (at most seg blocks unless one run is longer)
            std::vector<int32_t> ls;
            for (int64_t b = b0; b < b1; ++b) ls.push_back(bt[4 * b + 3]);
            std::sort(ls.begin(), ls.end());
            ls.erase(std::unique(ls.begin(), ls.end()), ls.end());
            for (size_t c0 = 0; c0 < ls.size(); c0 += (size_t)band) {
                const size_t c1 = std::min(ls.size(), c0 + (size_t)band);
                std::vector<int32_t> blk;
                for (int64_t b = b0; b < b1; ++b) {
                    const int32_t L = bt[4 * b + 3];
                    if (L >= ls[c0] && L <= ls[c1 - 1]) blk.push_back((int32_t)b);
                }
                size_t r0 = 0;
                while (r0 < blk.size()) {
                    size_t r1 = r0;
                    while (r1 < blk.size()) {
                        size_t rn = r1;  // end of the K-run starting at r1
                        while (rn < blk.size() && bt[4 * blk[rn] + 2] == bt[4 * blk[r1] + 2]) ++rn;
                        if (r1 > r0 && rn - r0 > (size_t)seg) break;
                        r1 = rn;
                    }
                    WorkItem it{(int32_t)entries.size(), (int32_t)(entries.size() + (r1 - r0)), I, J, 2, 0, -1, 0};
                    for (size_t r = r0; r < r1; ++r) entries.push_back(blk[r]);
                    groups.back().push_back(it);
                    r0 = r1;
                }
            }
        }
        b0 = b1;
    }
    wp.items = interleave(groups, xcd);
    std::vector<int32_t>& eslot = wp.eslot;
    eslot.assign((size_t)kSlotFields * std::max<size_t>(entries.size(), 1), -1);
    // Partial slots in creation order, item by item: K slots per run (targets
    // (I, key), (J, key)); J: visit 0 and fused one per item (target (I, J)),
    // visit 1 and fused one per entry (target (K, L)); fused L slots per band
    // position used in the item (targets (I, L), (J, L)).  A fused entry's
    // band position is the rank of its L among the item's L values in the
    // order they first occur: the index of the item's accumulator pair.
    std::vector<int64_t> ktgt, jtgt;
    for (WorkItem& it : wp.items) {
        int prev = -1;
        int32_t ka = -1, kb = -1;
        int32_t la[kMaxBand], lb[kMaxBand], lval[kMaxBand];
        int nl = 0;
        if (it.visit != 1) {
            it.jslot0 = (int32_t)jtgt.size();
            jtgt.push_back((int64_t)it.I * T + it.J);
        }
        for (int32_t e = it.e0; e < it.e1; ++e) {
            const int32_t b = entries[e];
            const int32_t K = bt[4 * b + 2], L = bt[4 * b + 3];
            const int key = it.visit == 1 ? L : K;
            if (key != prev) {
                ka = (int32_t)ktgt.size();
                ktgt.push_back((int64_t)it.I * T + key);
                kb = (int32_t)ktgt.size();
                ktgt.push_back((int64_t)it.J * T + key);
                prev = key;
            }
            int32_t* es = &eslot[(size_t)kSlotFields * e];
            es[kSlotKA] = ka;
            es[kSlotKB] = kb;
            if (it.visit != 0) {
                es[kSlotJ] = (int32_t)jtgt.size();
                jtgt.push_back((int64_t)K * T + L);
            }
            if (it.visit == 2) {
                int p = 0;
                while (p < nl && lval[p] != L) ++p;
                if (p == nl) {
                    if (nl >= band) return -1;  // cannot happen: an item spans one band
                    lval[nl] = L;
                    la[nl] = (int32_t)ktgt.size();
                    ktgt.push_back((int64_t)it.I * T + L);
                    lb[nl] = (int32_t)ktgt.size();
                    ktgt.push_back((int64_t)it.J * T + L);
                    ++nl;
                }
                es[kSlotLA] = la[p];
                es[kSlotLB] = lb[p];
                es[kSlotBpos] = p;
            }
        }
        if (ktgt.size() > (size_t)INT32_MAX / 2 || jtgt.size() > (size_t)INT32_MAX / 2) return -1;
    }
    wp.nkslots = (int64_t)ktgt.size();
    wp.njslots = (int64_t)jtgt.size();
    std::vector<int32_t> knew, jnew;
    renumber(ktgt, (int64_t)T * T, wp.kptr, knew);
    renumber(jtgt, (int64_t)T * T, wp.jptr, jnew);
    for (size_t e = 0; e < entries.size(); ++e) {
        int32_t* es = &eslot[(size_t)kSlotFields * e];
        for (int f : {(int)kSlotKA, (int)kSlotKB, (int)kSlotLA, (int)kSlotLB})
            if (es[f] >= 0) es[f] = knew[(size_t)es[f]];
        if (es[kSlotJ] >= 0) es[kSlotJ] = jnew[(size_t)es[kSlotJ]];
    }
    for (WorkItem& it : wp.items)
        if (it.jslot0 >= 0) it.jslot0 = jnew[(size_t)it.jslot0];
    // tile pairs read as operands: X_JL, X_IL, X_JK, X_IK and S_KL, S_IJ
    {
        std::vector<uint8_t> mark((size_t)T * T, 0);
        for (int64_t b = 0; b < nb; ++b) {
            const int I = bt[4 * b], J = bt[4 * b + 1], K = bt[4 * b + 2], L = bt[4 * b + 3];
            mark[(size_t)J * T + L] = mark[(size_t)I * T + L] = 1;
            mark[(size_t)J * T + K] = mark[(size_t)I * T + K] = 1;
            mark[(size_t)K * T + L] = mark[(size_t)I * T + J] = 1;
        }
        for (size_t x = 0; x < mark.size(); ++x)
            if (mark[x]) wp.used.push_back((int32_t)x);
    }
    // unordered tile pairs that receive partials (the reduction's work list)
    for (int X = 0; X < T; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            const size_t xy = (size_t)X * T + Y, yx = (size_t)Y * T + X;
            if (wp.kptr[xy + 1] > wp.kptr[xy] || wp.kptr[yx + 1] > wp.kptr[yx] || wp.jptr[xy + 1] > wp.jptr[xy])
                wp.red.push_back((int32_t)xy);
        }
    return 0;
}

}  // namespace esmf
