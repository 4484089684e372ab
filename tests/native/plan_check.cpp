// Test driver of the host planner (paper_2002_00322_amd/csrc/plan.cpp): reads
// a molecule, its Schwarz factors in function order and the plan settings
// from a binary file, runs the tile plan, the block list and one work plan,
// and writes every array the device launch consumes to a binary file, for
// the checks in tests/test_plan_cpu.py.  Built with g++ (optionally with
// sanitizers); no device code.
//
// input:  int32 nbf, kind, seg, band, xcd; float64 tau; float64 centers[nbf][3],
//         exponents[nbf], q[nbf][nbf]
// output: a sequence of arrays, each int64 count then the values: slot_fn
//         (i32), blk_tiles (i32), weight (f64), entries (i32), items (i32, 8 per
//         item), eslot (i32), kptr (i64), jptr (i64), used (i32), red (i32),
//         then int64 nkslots, njslots, int32 return code of plan_work
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "plan.h"

using namespace esmf;

template <typename T>
static bool rd(FILE* f, T* p, size_t n) {
    return fread(p, sizeof(T), n, f) == n;
}

template <typename T>
static void wr(FILE* f, const std::vector<T>& v) {
    const int64_t n = (int64_t)v.size();
    fwrite(&n, sizeof n, 1, f);
    if (n) fwrite(v.data(), sizeof(T), v.size(), f);
}

int main(int argc, char** argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: plan_check IN OUT\n");
        return 2;
    }
    FILE* in = fopen(argv[1], "rb");
    if (!in) return 3;
    int32_t hdr[5];
    double tau = 0.0;
    if (!rd(in, hdr, 5) || !rd(in, &tau, 1)) return 4;
    const int n = hdr[0], kind = hdr[1], seg = hdr[2], band = hdr[3], xcd = hdr[4];
    if (n < 1 || n > 4096) return 5;
    std::vector<double> centers(3 * (size_t)n), alpha(n), qf((size_t)n * n);
    if (!rd(in, centers.data(), centers.size()) || !rd(in, alpha.data(), alpha.size()) ||
        !rd(in, qf.data(), qf.size()))
        return 6;
    fclose(in);
    const std::vector<int32_t> slot_fn = make_tile_plan(n, centers.data(), alpha.data());
    const size_t ns = slot_fn.size();
    std::vector<double> qs(ns * ns, 0.0);
    for (size_t a = 0; a < ns; ++a)
        for (size_t b = 0; b < ns; ++b)
            if (slot_fn[a] >= 0 && slot_fn[b] >= 0) qs[a * ns + b] = qf[(size_t)slot_fn[a] * n + slot_fn[b]];
    BlockList bl;
    plan_blocks(qs, slot_fn, tau, bl);
    WorkPlan wp;
    const int32_t rc = plan_work(bl, kind, seg, band, xcd, wp);
    std::vector<int32_t> items;
    for (const WorkItem& it : wp.items) {
        const int32_t x[8] = {it.e0, it.e1, it.I, it.J, it.visit, it.reserved, it.jslot0, it.unit};
        items.insert(items.end(), x, x + 8);
    }
    FILE* out = fopen(argv[2], "wb");
    if (!out) return 7;
    wr(out, bl.slot_fn);
    wr(out, bl.blk_tiles);
    wr(out, bl.weight);
    wr(out, wp.entries);
    wr(out, items);
    wr(out, wp.eslot);
    wr(out, wp.kptr);
    wr(out, wp.jptr);
    wr(out, wp.used);
    wr(out, wp.red);
    fwrite(&wp.nkslots, sizeof(int64_t), 1, out);
    fwrite(&wp.njslots, sizeof(int64_t), 1, out);
    fwrite(&rc, sizeof rc, 1, out);
    fclose(out);
    return 0;
}
