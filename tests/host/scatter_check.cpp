// Host check of the scatter tables (no GPU): for plan p (step 2 of the
// batched corner chain) and plan q (step 3, whose A operand is p's output),
// every product of p's groups must land, through the tables, on the A-panel
// position that q's gather of the stored product would copy it to, and no
// other product may land anywhere.  Returns the number of products checked,
// or a negative code naming the first failure.
#include <vector>

#include "internal.hpp"

struct symten_tensor {
    symten::TensorPtr t;
};

extern "C" long long scatter_check(symten_tensor* A2, symten_tensor* B2, symten_tensor* B3, int prec) {
    using namespace symten;
    const int la2[1] = {0}, lb2[1] = {2}, la3[2] = {3, 1}, lb3[2] = {0, 1};
    auto p = plan_contraction(*A2->t, *B2->t, 1, la2, lb2, nullptr, prec);
    auto q = plan_contraction(*p->out_meta, *B3->t, 2, la3, lb3, nullptr, prec);
    std::vector<GemmGroup> groups(p->groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        groups[g] = GemmGroup{};
        groups[g].M = p->groups[g].M;
        groups[g].N = p->groups[g].N;
    }
    std::vector<int> tab;
    const int64_t written = append_scatter_tables(*p, *A2->t, *B2->t, *q, 0, groups.data(), tab);
    validate_scatter(groups, tab, std::max<int64_t>(q->a_panel_elems, 1), 1);
    // where q's gather puts each element of p's output
    std::vector<int64_t> dst(p->out_elems, -1);
    int64_t covered = 0;
    for (const CopyTask& t : q->copies) {
        if (t.src_buf != 0) continue;
        for (int64_t e = 0; e < t.count; ++e) {
            int64_t so = t.src_off, d = t.dst_off, r = e;
            for (int k = t.rank - 1; k >= 0; --k) {
                const int64_t ik = r % t.dims[k];
                r /= t.dims[k];
                so += ik * t.sstride[k];
                d += ik * t.dstride[k];
            }
            if (dst[so] != -1) return -1;   // an element gathered twice
            dst[so] = d;
            ++covered;
        }
    }
    if (covered != written) return -2;
    int64_t checked = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const GemmGroup& G = groups[gi];
        for (int i = 0; i < G.M; ++i)
            for (int j = 0; j < G.N; ++j) {
                const int* rr = &tab[G.s_rows + 4 * i];
                const int* cr = &tab[G.s_cols + 4 * j];
                const int* b = &tab[G.s_blocks + 8 * ((int64_t)rr[0] * G.s_ncb + cr[0])];
                const int64_t d = b[0] < 0 ? -1
                                           : (int64_t)b[0] + (int64_t)rr[1] * b[1] + (int64_t)rr[2] * b[2] +
                                                 (int64_t)rr[3] * b[3] + (int64_t)cr[1] * b[4] +
                                                 (int64_t)cr[2] * b[5] + (int64_t)cr[3] * b[6];
                if (d != dst[p->groups[gi].c_off + (int64_t)i * G.N + j]) return -3;
                checked += d >= 0;
            }
    }
    return checked == covered ? checked : -4;
}
