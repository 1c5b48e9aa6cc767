// Host-side planner (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <array>

namespace strassen {
namespace {

// One level of Strassen as coefficient vectors over the four quadrants
// (quadrant q = 2*row_half + col_half: 0 top-left, 1 top-right, 2 bottom-left,
// 3 bottom-right; eq. strassenpart).  Row i is product M_i of eq. gpu_allops:
//   M_i = (sum_q U[i][q] A_q) (sum_q V[i][q] B_q),   C_q += W[i][q] M_i.
constexpr int U[7][4] = {
    {1, 0, 0, 1},    // M0: A0 + A3
    {0, 0, 1, 1},    // M1: A2 + A3
    {1, 0, 0, 0},    // M2: A0
    {0, 0, 0, 1},    // M3: A3
    {1, 1, 0, 0},    // M4: A0 + A1
    {-1, 0, 1, 0},   // M5: A2 - A0
    {0, 1, 0, -1},   // M6: A1 - A3
};
constexpr int V[7][4] = {
    {1, 0, 0, 1},    // M0: B0 + B3
    {1, 0, 0, 0},    // M1: B0
    {0, 1, 0, -1},   // M2: B1 - B3
    {-1, 0, 1, 0},   // M3: B2 - B0
    {0, 0, 0, 1},    // M4: B3
    {1, 1, 0, 0},    // M5: B0 + B1
    {0, 0, 1, 1},    // M6: B2 + B3
};
constexpr int W[7][4] = {
    {1, 0, 0, 1},    // M0 -> C0, C3
    {0, 0, 1, -1},   // M1 -> C2, -C3
    {0, 1, 0, 1},    // M2 -> C1, C3
    {1, 0, 1, 0},    // M3 -> C0, C2
    {-1, 1, 0, 0},   // M4 -> -C0, C1
    {0, 0, 0, 1},    // M5 -> C3
    {1, 0, 0, 0},    // M6 -> C0
};

// Refines the terms of a d x d partition by one quadrant level with
// coefficients coef[4]: block (R, Cc) becomes blocks (2R + q/2, 2Cc + q%2).
int refine(const Term *in, int nin, int d, const int coef[4], Term *out) {
    int n = 0;
    for (int t = 0; t < nin; ++t) {
        const int R = in[t].block / d, Cc = in[t].block % d;
        for (int q = 0; q < 4; ++q) {
            if (coef[q] == 0) continue;
            const int r2 = 2 * R + q / 2, c2 = 2 * Cc + q % 2;
            out[n].block = r2 * (2 * d) + c2;
            out[n].sign = in[t].sign * coef[q];
            ++n;
        }
    }
    return n;
}

bool c_disjoint(const Product &x, const Product &y) {
    for (int i = 0; i < x.nc; ++i)
        for (int j = 0; j < y.nc; ++j)
            if (x.c[i].block == y.c[j].block) return false;
    return true;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

}  // namespace

std::vector<Product> scheme(int levels) {
    std::vector<Product> cur(1);
    cur[0].na = cur[0].nb = cur[0].nc = 1;
    cur[0].a[0] = cur[0].b[0] = cur[0].c[0] = Term{0, 1};
    int d = 1;
    for (int l = 0; l < levels; ++l) {
        std::vector<Product> next;
        next.reserve(cur.size() * 7);
        for (const Product &p : cur) {
            for (int i = 0; i < 7; ++i) {
                Product r;
                r.na = refine(p.a, p.na, d, U[i], r.a);
                r.nb = refine(p.b, p.nb, d, V[i], r.b);
                r.nc = refine(p.c, p.nc, d, W[i], r.c);
                next.push_back(r);
            }
        }
        cur.swap(next);
        d *= 2;
    }
    return cur;
}

std::vector<StreamSlot> stream_stages() {
    // stage 0: M1, M5 on stream 0 and M4, M6 on stream 1 (M1 and M5 share
    // C3, M4 and M6 share C0); stage 1: M2 | M3; stage 2: M0.
    return {{1, 0, 0}, {5, 0, 0}, {4, 0, 1}, {6, 0, 1}, {2, 1, 0}, {3, 1, 1}, {0, 2, 0}};
}

Plan make_plan(int64_t m, int64_t n, int64_t k, int levels, int vec, bool round_m) {
    Plan p;
    p.levels = levels;
    p.d = 1 << levels;
    p.m = m;
    p.n = n;
    p.k = k;
    p.sm = ceil_div(m, p.d);
    p.sn = ceil_div(n, p.d);
    p.sk = ceil_div(k, p.d);
    if (levels > 0 && vec > 1) {
        p.sn = round_up(p.sn, vec);
        p.sk = round_up(p.sk, vec);
        if (round_m) p.sm = round_up(p.sm, vec);
    }
    const std::vector<Product> all = scheme(levels);

    // Race-free batches (Task Parallelism section, batching by variant): a
    // batch holds products of one variant (W_A, W_B, W_C) whose C write sets
    // are pairwise disjoint, so one launch never has two workgroups updating
    // the same C element.  Greedy first fit in canonical order.
    std::vector<std::array<int, 3>> variants;
    for (const Product &q : all) {
        std::array<int, 3> v = {q.na, q.nb, q.nc};
        if (std::find(variants.begin(), variants.end(), v) == variants.end())
            variants.push_back(v);
    }
    for (const auto &v : variants) {
        const size_t first_batch = p.batches.size();
        for (int i = 0; i < (int)all.size(); ++i) {
            const Product &q = all[i];
            if (q.na != v[0] || q.nb != v[1] || q.nc != v[2]) continue;
            bool placed = false;
            for (size_t b = first_batch; b < p.batches.size() && !placed; ++b) {
                Batch &bt = p.batches[b];
                if ((int)bt.products.size() >= kMaxBatch) continue;
                bool ok = true;
                for (int j : bt.products) ok = ok && c_disjoint(all[j], q);
                if (ok) {
                    bt.products.push_back(i);
                    placed = true;
                }
            }
            if (!placed) p.batches.push_back(Batch{v[0], v[1], v[2], {i}});
        }
    }

    // Products in launch order; batches refer to positions in that order.
    for (Batch &bt : p.batches) {
        for (int &idx : bt.products) {
            p.products.push_back(all[idx]);
            idx = (int)p.products.size() - 1;
        }
    }

    // The first update of each C block in launch order applies beta.
    std::vector<bool> touched((size_t)p.d * p.d, false);
    for (Product &q : p.products)
        for (int o = 0; o < q.nc; ++o) {
            q.c_first[o] = !touched[q.c[o].block];
            touched[q.c[o].block] = true;
        }

    p.executed_flops = (double)p.products.size() * 2.0 * (double)p.sm *
                       (double)p.sn * (double)p.sk;
    return p;
}

}  // namespace strassen
