// SU(2) reduced tensors: canonical coupling-tree blocks and the contraction
// plan with recoupling scalars.
//
// A block carries one spin per leg and one coupling tree (Sec. 2, Eq.
// tensor-cgc: t_i = m_i (x) c_i).  Incoming legs are coupled left to right
// by Clebsch-Gordan coefficients to a total spin K, outgoing legs likewise
// to the same K; the tree labels are (in-chain intermediates, out-chain
// intermediates, K) and the block's generalised CGC tensor is
// c[m_1..m_R] = sum_M C_in(m_in; K M) C_out(m_out; K M).
//
// A contraction multiplies reduced blocks and CGC tensors separately (Sec. 2,
// contraction rule r_k = (m_t . m_s) (x) (c_t . c_s)); the product c_t . c_s
// is expanded in the canonical basis of the output legs, and every non-zero
// coefficient X becomes one scaled term of the output block's sector GEMM.
// The scalars are computed once per plan on the host in FP64.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>

#include "internal.hpp"

namespace symten {

// ------------------------------------------------------ Clebsch-Gordan
// <j1 m1; j2 m2 | J M>, arguments doubled, Condon-Shortley phase, from
// Racah's closed form (sum over k), in long double.
static long double lfact(int n) {
    static std::vector<long double> f = [] {
        std::vector<long double> v(200, 1.0L);
        for (int i = 1; i < 200; ++i) v[i] = v[i - 1] * i;
        return v;
    }();
    return f[n];
}

double cg_coeff(int tj1, int tm1, int tj2, int tm2, int tJ, int tM) {
    if (tm1 + tm2 != tM) return 0.0;
    if (tJ < std::abs(tj1 - tj2) || tJ > tj1 + tj2 || (tj1 + tj2 + tJ) % 2) return 0.0;
    if (std::abs(tm1) > tj1 || std::abs(tm2) > tj2 || std::abs(tM) > tJ) return 0.0;
    if ((tj1 + tm1) % 2 || (tj2 + tm2) % 2 || (tJ + tM) % 2) return 0.0;
    const int a = (tj1 + tj2 - tJ) / 2, b = (tj1 - tj2 + tJ) / 2, c = (-tj1 + tj2 + tJ) / 2;
    const int d = (tj1 + tj2 + tJ) / 2 + 1;
    const long double pre = std::sqrt((tJ + 1) * lfact(a) * lfact(b) * lfact(c) / lfact(d)) *
                            std::sqrt(lfact((tj1 + tm1) / 2) * lfact((tj1 - tm1) / 2) * lfact((tj2 + tm2) / 2) *
                                      lfact((tj2 - tm2) / 2) * lfact((tJ + tM) / 2) * lfact((tJ - tM) / 2));
    long double s = 0.0L;
    for (int k = 0; k <= d; ++k) {
        const int e1 = a - k, e2 = (tj1 - tm1) / 2 - k, e3 = (tj2 + tm2) / 2 - k;
        const int e4 = (tJ - tj2 + tm1) / 2 + k, e5 = (tJ - tj1 - tm2) / 2 + k;
        if (e1 < 0 || e2 < 0 || e3 < 0 || e4 < 0 || e5 < 0) continue;
        const long double den = lfact(k) * lfact(e1) * lfact(e2) * lfact(e3) * lfact(e4) * lfact(e5);
        s += ((k % 2) ? -1.0L : 1.0L) / den;
    }
    return (double)(pre * s);
}

// ------------------------------------------------------------ trees
static std::vector<std::vector<int>> chains(const std::vector<int>& tjs) {
    if (tjs.empty()) return {{0}};
    std::vector<std::vector<int>> out{{tjs[0]}};
    for (size_t i = 1; i < tjs.size(); ++i) {
        std::vector<std::vector<int>> nxt;
        for (auto& c : out) {
            const int k = c.back();
            for (int K = std::abs(k - tjs[i]); K <= k + tjs[i]; K += 2) {
                auto d = c;
                d.push_back(K);
                nxt.push_back(d);
            }
        }
        out.swap(nxt);
    }
    return out;
}

static void split_dirs(const std::vector<Leg>& legs, std::vector<int>& ins, std::vector<int>& outs) {
    ins.clear();
    outs.clear();
    for (size_t i = 0; i < legs.size(); ++i) (legs[i].dir > 0 ? ins : outs).push_back((int)i);
}

// all (tj tuple, tree) of the legs, canonical (lexicographic) order
static std::vector<std::pair<std::vector<int>, std::vector<int>>> su2_labels(const std::vector<Leg>& legs) {
    std::vector<int> ins, outs;
    split_dirs(legs, ins, outs);
    std::vector<std::pair<std::vector<int>, std::vector<int>>> res;
    const int R = (int)legs.size();
    std::vector<int> idx(R, 0);
    for (auto& l : legs)
        if (l.q.empty()) return res;
    while (true) {
        std::vector<int> tj(R);
        for (int l = 0; l < R; ++l) tj[l] = legs[l].q[idx[l]];
        std::vector<int> ti, to;
        for (int i : ins) ti.push_back(tj[i]);
        for (int o : outs) to.push_back(tj[o]);
        for (auto& a : chains(ti))
            for (auto& b : chains(to)) {
                if (a.back() != b.back()) continue;
                std::vector<int> tree;
                for (size_t k = 1; k + 1 < a.size(); ++k) tree.push_back(a[k]);
                for (size_t k = 1; k + 1 < b.size(); ++k) tree.push_back(b[k]);
                tree.push_back(a.back());
                res.push_back({tj, tree});
            }
        int l = R - 1;
        while (l >= 0 && ++idx[l] == (int)legs[l].q.size()) { idx[l] = 0; --l; }
        if (l < 0) break;
    }
    std::sort(res.begin(), res.end());
    return res;
}

int64_t enumerate_blocks_su2(Tensor& t) {
    t.blocks.clear();
    int64_t off = 0;
    for (auto& lt : su2_labels(t.legs)) {
        Block b;
        b.q = lt.first;
        b.tree = lt.second;
        const int R = t.rank();
        b.shape.resize(R);
        b.stride.resize(R);
        int64_t sz = 1;
        for (int l = 0; l < R; ++l) {
            b.shape[l] = t.legs[l].dim_of(b.q[l]);
            sz *= b.shape[l];
        }
        int64_t st = 1;
        for (int l = R - 1; l >= 0; --l) { b.stride[l] = st; st *= b.shape[l]; }
        b.offset = off;
        b.size = sz;
        off += sz;
        t.blocks.push_back(std::move(b));
    }
    t.rebuild_index();
    return off;
}

// ------------------------------------------------------- CGC tensors
namespace {
struct DenseT {
    std::vector<int> shape;   // (tj + 1) per leg
    std::vector<double> v;    // row-major
};

// C(m_1..m_r; K M) of one chain as [m_1..m_r][M]
std::vector<double> chain_tensor(const std::vector<int>& tjs, const std::vector<int>& chain, int K) {
    if (tjs.empty()) return {1.0};
    int64_t n = 1;
    for (int t : tjs) n *= t + 1;
    std::vector<double> C(n * (K + 1), 0.0);
    std::vector<int> mm(tjs.size());
    for (int64_t lin = 0; lin < n; ++lin) {
        int64_t r = lin;
        for (int i = (int)tjs.size() - 1; i >= 0; --i) {
            mm[i] = -tjs[i] + 2 * (int)(r % (tjs[i] + 1));
            r /= tjs[i] + 1;
        }
        double val = 1.0;
        int mu = mm[0];
        for (size_t s = 1; s < tjs.size() && val != 0.0; ++s) {
            const int nmu = mu + mm[s];
            val *= cg_coeff(chain[s - 1], mu, tjs[s], mm[s], chain[s], nmu);
            mu = nmu;
        }
        if (val != 0.0 && std::abs(mu) <= K) C[lin * (K + 1) + (mu + K) / 2] = val;
    }
    return C;
}

DenseT cgc_tensor(const std::vector<Leg>& legs, const std::vector<int>& tj, const std::vector<int>& tree) {
    std::vector<int> ins, outs;
    split_dirs(legs, ins, outs);
    const int K = tree.back();
    const size_t nim = ins.size() >= 2 ? ins.size() - 2 : 0;
    const size_t nom = outs.size() >= 2 ? outs.size() - 2 : 0;
    auto make_chain = [&](const std::vector<int>& tjs, size_t from, size_t cnt) {
        if (tjs.empty()) return std::vector<int>{0};
        if (tjs.size() == 1) return std::vector<int>{tjs[0]};
        std::vector<int> c{tjs[0]};
        for (size_t k = 0; k < cnt; ++k) c.push_back(tree[from + k]);
        c.push_back(K);
        return c;
    };
    std::vector<int> ti, to;
    for (int i : ins) ti.push_back(tj[i]);
    for (int o : outs) to.push_back(tj[o]);
    const std::vector<double> Ci = chain_tensor(ti, make_chain(ti, 0, nim), K);
    const std::vector<double> Co = chain_tensor(to, make_chain(to, nim, nom), K);
    const int64_t ni = (int64_t)Ci.size() / (K + 1), no = (int64_t)Co.size() / (K + 1);
    DenseT c;
    const int R = (int)legs.size();
    c.shape.resize(R);
    for (int l = 0; l < R; ++l) c.shape[l] = tj[l] + 1;
    c.v.assign(ni * no, 0.0);
    // strides of the (ins..., outs...) order inside the leg-order tensor
    std::vector<int64_t> st(R);
    int64_t s = 1;
    for (int l = R - 1; l >= 0; --l) { st[l] = s; s *= c.shape[l]; }
    std::vector<int> order = ins;
    order.insert(order.end(), outs.begin(), outs.end());
    for (int64_t a = 0; a < ni; ++a)
        for (int64_t b = 0; b < no; ++b) {
            double v = 0.0;
            for (int M = 0; M <= K; ++M) v += Ci[a * (K + 1) + M] * Co[b * (K + 1) + M];
            if (v == 0.0) continue;
            // decode (a over ins, b over outs) into the leg-order index
            int64_t lin = 0, ra = a, rb = b;
            for (int k = (int)ins.size() - 1; k >= 0; --k) {
                lin += (ra % c.shape[ins[k]]) * st[ins[k]];
                ra /= c.shape[ins[k]];
            }
            for (int k = (int)outs.size() - 1; k >= 0; --k) {
                lin += (rb % c.shape[outs[k]]) * st[outs[k]];
                rb /= c.shape[outs[k]];
            }
            c.v[lin] = v;
        }
    return c;
}

std::mutex g_cgc_mu;
std::map<std::vector<int>, DenseT> g_cgc;   // key: dirs, tj, tree

const DenseT& cgc_cached(const std::vector<Leg>& legs, const std::vector<int>& tj, const std::vector<int>& tree) {
    std::vector<int> key;
    for (auto& l : legs) key.push_back(l.dir);
    key.push_back(1000);
    key.insert(key.end(), tj.begin(), tj.end());
    key.push_back(1000);
    key.insert(key.end(), tree.begin(), tree.end());
    std::lock_guard<std::mutex> lk(g_cgc_mu);
    auto it = g_cgc.find(key);
    if (it != g_cgc.end()) return it->second;
    return g_cgc.emplace(key, cgc_tensor(legs, tj, tree)).first->second;
}

// P[free_a..., free_b...] = sum over contracted m of cA * cB
DenseT contract_cgc(const DenseT& ca, const DenseT& cb, const std::vector<int>& conA, const std::vector<int>& conB,
                    const std::vector<int>& freeA, const std::vector<int>& freeB) {
    DenseT p;
    for (int l : freeA) p.shape.push_back(ca.shape[l]);
    for (int l : freeB) p.shape.push_back(cb.shape[l]);
    int64_t nfa = 1, nfb = 1, nk = 1;
    for (int l : freeA) nfa *= ca.shape[l];
    for (int l : freeB) nfb *= cb.shape[l];
    for (int l : conA) nk *= ca.shape[l];
    auto strides = [](const std::vector<int>& shape) {
        std::vector<int64_t> st(shape.size());
        int64_t s = 1;
        for (int l = (int)shape.size() - 1; l >= 0; --l) { st[l] = s; s *= shape[l]; }
        return st;
    };
    const std::vector<int64_t> sa = strides(ca.shape), sb = strides(cb.shape);
    auto offsets = [](const std::vector<int>& legs, const std::vector<int>& shape, const std::vector<int64_t>& st) {
        int64_t n = 1;
        for (int l : legs) n *= shape[l];
        std::vector<int64_t> off(n, 0);
        for (int64_t i = 0; i < n; ++i) {
            int64_t r = i, o = 0;
            for (int k = (int)legs.size() - 1; k >= 0; --k) {
                o += (r % shape[legs[k]]) * st[legs[k]];
                r /= shape[legs[k]];
            }
            off[i] = o;
        }
        return off;
    };
    const auto ofa = offsets(freeA, ca.shape, sa), oka = offsets(conA, ca.shape, sa);
    const auto ofb = offsets(freeB, cb.shape, sb), okb = offsets(conB, cb.shape, sb);
    p.v.assign(nfa * nfb, 0.0);
    for (int64_t i = 0; i < nfa; ++i)
        for (int64_t k = 0; k < nk; ++k) {
            const double x = ca.v[ofa[i] + oka[k]];
            if (x == 0.0) continue;
            for (int64_t j = 0; j < nfb; ++j) p.v[i * nfb + j] += x * cb.v[ofb[j] + okb[k]];
        }
    return p;
}
}  // namespace

// -------------------------------------------------------------- planning
namespace {
std::vector<int64_t> suffix_strides(const std::vector<int>& d, int64_t mult) {
    std::vector<int64_t> s(d.size());
    int64_t st = mult;
    for (int k = (int)d.size() - 1; k >= 0; --k) { s[k] = st; st *= d[k]; }
    return s;
}

// <c_o, P> / <c_o, c_o> where P is laid out in the unpermuted output order
// and c_o in the permuted one (out leg j is unpermuted leg perm[j]).
double project(const DenseT& co, const DenseT& pr, const std::vector<int>& perm) {
    const int RO = (int)perm.size();
    std::vector<int64_t> st_un(RO);
    int64_t s = 1;
    for (int l = RO - 1; l >= 0; --l) { st_un[l] = s; s *= pr.shape[l]; }
    double num = 0.0, den = 0.0;
    std::vector<int> idx(RO, 0);
    const int64_t n = (int64_t)co.v.size();
    for (int64_t lin = 0; lin < n; ++lin) {
        const double cv = co.v[lin];
        if (cv != 0.0) {
            int64_t o = 0;
            for (int j = 0; j < RO; ++j) o += idx[j] * st_un[perm[j]];
            num += cv * pr.v[o];
            den += cv * cv;
        }
        for (int j = RO - 1; j >= 0; --j) {
            if (++idx[j] < co.shape[j]) break;
            idx[j] = 0;
        }
    }
    return den > 0.0 ? num / den : 0.0;
}
}  // namespace

// Reduced contraction (Sec. 2, Eq. contraction rule with CGCs): every matched
// pair (A block, B block) contributes (m_A . m_B) x (c_A . c_B); the CGC
// product is expanded in the canonical basis of the output legs,
// c_A . c_B = sum_b X_b c_b, and each X_b != 0 adds X_b m_A . m_B to output
// block b.  All terms of one output block form one GEMM: the K ranges of the
// terms are concatenated, the A panel of a term carries X_b.  Scalars whose
// magnitude is below 1e-13 are structural zeros and are dropped.
std::shared_ptr<ContractPlan> plan_contraction_su2(const Tensor& A, const Tensor& B, const std::vector<int>& conA,
                                                   const std::vector<int>& conB, const std::vector<int>& freeA,
                                                   const std::vector<int>& freeB, const std::vector<int>& perm,
                                                   Prec p) {
    const int RO = (int)perm.size();
    auto plan = std::make_shared<ContractPlan>();
    plan->prec = p;
    plan->panel_f64 = p == Prec::F64;
    const int VW = panel_vw(p);

    auto out = std::make_shared<Tensor>();
    out->group = SYMTEN_SU2;
    out->flux = 0;
    out->dtype = A.dtype;
    std::vector<Leg> olegs;   // unpermuted order: A free legs, then B free legs
    for (int l : freeA) olegs.push_back(A.legs[l]);
    for (int l : freeB) olegs.push_back(B.legs[l]);
    out->legs.resize(RO);
    for (int j = 0; j < RO; ++j) out->legs[j] = olegs[perm[j]];
    const auto olabels = su2_labels(out->legs);
    std::map<std::vector<int>, std::vector<int>> trees_of;   // output spins -> canonical block ids
    for (size_t i = 0; i < olabels.size(); ++i) trees_of[olabels[i].first].push_back((int)i);

    // B blocks by contracted spins
    std::map<std::vector<int>, std::vector<int>> b_by_con;
    for (size_t ib = 0; ib < B.blocks.size(); ++ib) {
        std::vector<int> k;
        for (int c : conB) k.push_back(B.blocks[ib].q[c]);
        b_by_con[k].push_back((int)ib);
    }

    struct Term { int a, b; double x; };
    std::map<int, std::vector<Term>> terms;   // canonical output block -> terms
    for (size_t ia = 0; ia < A.blocks.size(); ++ia) {
        const Block& ba = A.blocks[ia];
        std::vector<int> k;
        for (int c : conA) k.push_back(ba.q[c]);
        auto hit = b_by_con.find(k);
        if (hit == b_by_con.end()) continue;
        const DenseT& ca = cgc_cached(A.legs, ba.q, ba.tree);
        for (int ib : hit->second) {
            const Block& bb = B.blocks[ib];
            std::vector<int> tj_un;
            for (int l : freeA) tj_un.push_back(ba.q[l]);
            for (int l : freeB) tj_un.push_back(bb.q[l]);
            std::vector<int> tj(RO);
            for (int j = 0; j < RO; ++j) tj[j] = tj_un[perm[j]];
            auto ot = trees_of.find(tj);
            if (ot == trees_of.end()) continue;
            const DenseT& cb = cgc_cached(B.legs, bb.q, bb.tree);
            const DenseT pr = contract_cgc(ca, cb, conA, conB, freeA, freeB);
            for (int ob : ot->second) {
                const double x = project(cgc_cached(out->legs, tj, olabels[ob].second), pr, perm);
                if (std::fabs(x) > 1e-13) terms[ob].push_back({(int)ia, ib, x});
            }
        }
    }

    symten_plan_stats info{};
    int64_t a_pos = 0, b_pos = 0, c_pos = 0;
    auto align32 = [](int64_t x) { return (x + 31) / 32 * 32; };
    for (auto& kv : terms) {
        const auto& lab = olabels[kv.first];
        const std::vector<Term>& tl = kv.second;
        const Block& ba0 = A.blocks[tl[0].a];
        const Block& bb0 = B.blocks[tl[0].b];
        std::vector<int> adims, bdims;
        for (int l : freeA) adims.push_back(ba0.shape[l]);
        for (int l : freeB) bdims.push_back(bb0.shape[l]);
        int64_t M = 1, N = 1;
        for (int d : adims) M *= d;
        for (int d : bdims) N *= d;
        // K segments.  A-major: one segment per distinct A block, whose B
        // panel is the sum over that block's terms of x * B block (blocks that
        // differ in their tree only, same shape); B-major: the mirror image.
        // The layout with the smaller K is taken.  Sources of one segment
        // must share strides and number at most 1 + kMaxExtraSrc.
        struct Seg {
            int major;                                  // block of the major side
            std::vector<std::pair<int, double>> minor;  // (block, scalar) summed on the other side
            int64_t k;
        };
        auto segments = [&](bool a_major) {
            const Tensor& Mj = a_major ? A : B;
            const Tensor& Mn = a_major ? B : A;
            const std::vector<int>& conM = a_major ? conA : conB;
            std::map<int, std::vector<std::pair<int, double>>> by;
            for (auto& t : tl) (a_major ? by[t.a] : by[t.b]).push_back({a_major ? t.b : t.a, t.x});
            std::vector<Seg> out;
            for (auto& e : by) {
                int64_t k = 1;
                for (int c : conM) k *= Mj.blocks[e.first].shape[c];
                Seg cur{e.first, {}, k};
                for (auto& m : e.second) {
                    const bool fits = cur.minor.empty() ||
                                      ((int)cur.minor.size() <= kMaxExtraSrc &&
                                       Mn.blocks[m.first].stride == Mn.blocks[cur.minor[0].first].stride);
                    if (!fits) {
                        out.push_back(cur);
                        cur.minor.clear();
                    }
                    cur.minor.push_back(m);
                }
                out.push_back(cur);
            }
            return out;
        };
        const std::vector<Seg> seg_a = segments(true), seg_b = segments(false);
        int64_t ka = 0, kb = 0;
        for (auto& g : seg_a) ka += g.k;
        for (auto& g : seg_b) kb += g.k;
        const bool a_major = ka <= kb;
        const std::vector<Seg>& segs = a_major ? seg_a : seg_b;
        const int64_t K = a_major ? ka : kb;
        if (M == 0 || N == 0 || K == 0) continue;
        if (M >= (1LL << 31) || N >= (1LL << 31) || K >= (1LL << 30)) fail(SYMTEN_E_CAPACITY, "contract: sector too large");
        const int64_t lda = (K + VW - 1) / VW * VW;
        GroupPlan gp;
        gp.key = kv.first;
        gp.M = (int)M;
        gp.N = (int)N;
        gp.K = (int)K;
        gp.lda = (int)lda;
        gp.a_off = a_pos;
        gp.b_off = b_pos;
        gp.c_off = c_pos;
        a_pos = align32(a_pos + M * lda);
        b_pos = align32(b_pos + N * lda);
        c_pos += M * N;
        info.groups += 1;
        info.gemm_flops += 2 * M * N * K;
        info.useful_flops += 2 * M * N * K;
        info.pairs += (int64_t)tl.size();
        info.max_m = std::max<int64_t>(info.max_m, M);
        info.max_n = std::max<int64_t>(info.max_n, N);
        info.max_k = std::max<int64_t>(info.max_k, K);
        // panel task of one side: [free..., contracted...] of the listed blocks,
        // summed with their scalars, into columns koff.. of the panel rows
        auto panel_task = [&](const Tensor& X, const std::vector<int>& fr, const std::vector<int>& co,
                              const std::vector<int>& fdims, int src, int dst, int64_t doff,
                              const std::vector<std::pair<int, double>>& srcs) {
            const Block& b0 = X.blocks[srcs[0].first];
            std::vector<int> dims, kd;
            std::vector<int64_t> ss;
            for (int l : fr) { dims.push_back(b0.shape[l]); ss.push_back(b0.stride[l]); }
            for (int l : co) { dims.push_back(b0.shape[l]); ss.push_back(b0.stride[l]); kd.push_back(b0.shape[l]); }
            std::vector<int64_t> ds = suffix_strides(fdims, lda), dk = suffix_strides(kd, 1);
            ds.insert(ds.end(), dk.begin(), dk.end());
            CopyTask t = make_copy_task(src, b0.offset, dst, doff, dims, ss, ds, srcs[0].second);
            t.nextra = (int)srcs.size() - 1;
            for (int x = 1; x < (int)srcs.size(); ++x) {
                t.xsrc_off[x - 1] = X.blocks[srcs[x].first].offset;
                t.xscale[x - 1] = srcs[x].second;
            }
            plan->copies.push_back(t);
        };
        int64_t koff = 0;
        for (const Seg& g : segs) {
            const std::vector<std::pair<int, double>> major{{g.major, 1.0}};
            panel_task(A, freeA, conA, adims, 0, 2, gp.a_off + koff, a_major ? major : g.minor);
            panel_task(B, freeB, conB, bdims, 1, 3, gp.b_off + koff, a_major ? g.minor : major);
            koff += g.k;
        }
        if (lda > K) {
            plan->copies.push_back(make_copy_task(-1, 0, 2, gp.a_off + K, {(int)M, (int)(lda - K)}, {0, 0}, {lda, 1}));
            plan->copies.push_back(make_copy_task(-1, 0, 3, gp.b_off + K, {(int)N, (int)(lda - K)}, {0, 0}, {lda, 1}));
        }
        // output block: row-major [A free..., B free...] = M x N, seen through the permutation
        Block ob;
        ob.q = lab.first;
        ob.tree = lab.second;
        std::vector<int> shp = adims;
        shp.insert(shp.end(), bdims.begin(), bdims.end());
        std::vector<int64_t> st = suffix_strides(adims, N), sb = suffix_strides(bdims, 1);
        st.insert(st.end(), sb.begin(), sb.end());
        ob.shape.resize(RO);
        ob.stride.resize(RO);
        for (int j = 0; j < RO; ++j) {
            ob.shape[j] = shp[perm[j]];
            ob.stride[j] = st[perm[j]];
        }
        ob.offset = gp.c_off;
        ob.size = M * N;
        out->blocks.push_back(std::move(ob));
        info.out_blocks += 1;
        plan->groups.push_back(std::move(gp));
    }
    // canonical order (terms is keyed by the canonical index, so already sorted)
    out->rebuild_index();
    out->elems = c_pos;
    out->meta_only = true;
    plan->out_meta = out;
    plan->a_panel_elems = a_pos;
    plan->b_panel_elems = b_pos;
    plan->out_elems = c_pos;
    plan->info = info;
    if (panel_planes(p) > 1)
        for (auto& t : plan->copies) t.lo_off = t.dst_buf == 2 ? a_pos : b_pos;
    return plan;
}

// ------------------------------------------------------- S^z expansion
// t[(a_1, m_1), ..] = sum over the trees of the spin tuple of
// m_tree[a_1, ..] c_tree[m_1, ..] (Sec. 2, Eq. tensor-cgc), written into the
// U(1) blocks of charges (m_1, ..).  The trees of one spin tuple touch the same
// elements, so the gathers run in layers (layer t = t-th tree of every spin
// tuple), each accumulating onto the zeroed output.
TensorPtr su2_to_u1(const Tensor& in, hipStream_t stream) {
    if (in.group != SYMTEN_SU2) fail(SYMTEN_E_INVAL, "su2_to_u1: tensor is not SU(2)");
    check_device_tensor(in, "su2_to_u1");
    const int R = in.rank();
    auto out = std::make_shared<Tensor>();
    out->group = SYMTEN_U1;
    out->flux = 0;
    out->dtype = in.dtype;
    // per leg: (tj, m) -> position of multiplet 0 of spin tj inside charge m
    std::vector<std::map<std::pair<int, int>, int>> pos(R);
    for (int l = 0; l < R; ++l) {
        const Leg& L = in.legs[l];
        int tmax = 0;
        for (int t : L.q) tmax = std::max(tmax, t);
        Leg U;
        U.dir = L.dir;
        for (int m = -tmax; m <= tmax; ++m) {
            int d = 0;
            for (size_t i = 0; i < L.q.size(); ++i) {
                const int t = L.q[i];
                if (t >= std::abs(m) && (t - m) % 2 == 0) {
                    pos[l][{t, m}] = d;
                    d += L.d[i];
                }
            }
            if (d > 0) { U.q.push_back(m); U.d.push_back(d); }
        }
        out->legs.push_back(U);
    }
    out->elems = enumerate_blocks(*out);
    out->buf = device_alloc(std::max<int64_t>(out->elems, 1) * out->esize());
    out->meta_only = false;
    launch_fill_zero(out->buf->ptr, ((std::max<int64_t>(out->elems, 1) * out->esize() + 3) / 4) * 4, stream);

    std::vector<std::vector<CopyTask>> layers;
    std::map<std::vector<int>, int> layer_of;   // spins -> trees seen so far
    for (const Block& b : in.blocks) {
        if (b.size == 0) continue;
        const int layer = layer_of[b.q]++;
        if ((int)layers.size() <= layer) layers.resize(layer + 1);
        const DenseT& c = cgc_cached(in.legs, b.q, b.tree);
        std::vector<int> idx(R, 0);
        for (size_t lin = 0; lin < c.v.size(); ++lin) {
            if (c.v[lin] != 0.0) {
                std::vector<int> qs(R);
                for (int l = 0; l < R; ++l) qs[l] = -b.q[l] + 2 * idx[l];
                auto it = out->index.find(qs);
                if (it == out->index.end()) fail(SYMTEN_E_SYM, "su2_to_u1: CGC entry outside the U(1) blocks");
                const Block& ub = out->blocks[it->second];
                int64_t doff = ub.offset;
                for (int l = 0; l < R; ++l) doff += (int64_t)pos[l].at({b.q[l], qs[l]}) * ub.stride[l];
                layers[layer].push_back(make_copy_task(0, b.offset, 1, doff, b.shape, b.stride, ub.stride, c.v[lin]));
            }
            for (int l = R - 1; l >= 0; --l) {
                if (++idx[l] < c.shape[l]) break;
                idx[l] = 0;
            }
        }
    }
    const bool f64 = in.dtype == SYMTEN_F64;
    std::vector<BufferPtr> keep;
    for (auto& tasks : layers) {
        if (tasks.empty()) continue;
        validate_tasks(tasks, {in.elems, out->elems});
        std::vector<int64_t> prefix;
        copy_prefix(tasks, prefix);
        BufferPtr dt, dp;
        upload_sync(dt, tasks.data(), tasks.size() * sizeof(CopyTask));
        upload_sync(dp, prefix.data(), prefix.size() * sizeof(int64_t));
        copy_launch_arg((const CopyTask*)dt->ptr, (const int64_t*)dp->ptr, (int)tasks.size(), prefix.back(),
                        {in.data(), out->data()}, f64, /*accumulate*/ 4, stream);
        keep.push_back(dt);
        keep.push_back(dp);
    }
    // the descriptor buffers return to the pool when `keep` goes: wait first
    HIPCHK(hipStreamSynchronize(stream));
    return out;
}

// ------------------------------------------------- S^z basis helpers
namespace {
// S^z (U(1)) leg of an SU(2) leg: charges 2m; inside a charge the states run
// over spins ascending, then multiplets.  pos[(tj, m)] = first state of spin
// tj inside charge m; state_of[i] = (tj, multiplet, m) of U(1) state i.
struct SzLeg {
    Leg u1;
    std::map<std::pair<int, int>, int> pos;
    std::vector<std::array<int, 3>> state_of;
};
SzLeg sz_leg(const Leg& L) {
    SzLeg r;
    int tmax = 0;
    for (int t : L.q) tmax = std::max(tmax, t);
    r.u1.dir = L.dir;
    for (int m = -tmax; m <= tmax; ++m) {
        int d = 0;
        for (size_t i = 0; i < L.q.size(); ++i) {
            const int t = L.q[i];
            if (t >= std::abs(m) && (t - m) % 2 == 0) {
                r.pos[{t, m}] = d;
                for (int a = 0; a < L.d[i]; ++a) r.state_of.push_back({t, a, m});
                d += L.d[i];
            }
        }
        if (d > 0) { r.u1.q.push_back(m); r.u1.d.push_back(d); }
    }
    return r;
}
}  // namespace

TensorPtr u1_to_su2(const Tensor& U, const std::vector<Leg>& legs, hipStream_t stream) {
    if (U.group != SYMTEN_U1) fail(SYMTEN_E_INVAL, "u1_to_su2: tensor is not U(1)");
    check_device_tensor(U, "u1_to_su2");
    const int R = (int)legs.size();
    if (U.rank() != R) fail(SYMTEN_E_INVAL, "u1_to_su2: rank mismatch");
    std::vector<SzLeg> sz;
    for (int l = 0; l < R; ++l) {
        sz.push_back(sz_leg(legs[l]));
        if (sz[l].u1.dir != U.legs[l].dir || !sz[l].u1.same_sectors(U.legs[l]))
            fail(SYMTEN_E_LEGS, "u1_to_su2: U(1) legs are not the S^z legs of the SU(2) legs");
    }
    auto out = std::make_shared<Tensor>();
    out->group = SYMTEN_SU2;
    out->flux = 0;
    out->dtype = U.dtype;
    out->legs = legs;
    out->elems = enumerate_blocks_su2(*out);
    out->buf = device_alloc(std::max<int64_t>(out->elems, 1) * out->esize());
    out->meta_only = false;
    launch_fill_zero(out->buf->ptr, ((std::max<int64_t>(out->elems, 1) * out->esize() + 3) / 4) * 4, stream);
    // m[a..] = sum_m c[m] t[(a, m)..] / <c, c>: one accumulating gather per
    // non-zero basis-tensor entry; layer t holds the t-th entry of every block
    std::vector<std::vector<CopyTask>> layers;
    for (const Block& b : out->blocks) {
        if (b.size == 0) continue;
        const DenseT& c = cgc_cached(out->legs, b.q, b.tree);
        double nrm = 0.0;
        for (double v : c.v) nrm += v * v;
        std::vector<int> idx(R, 0);
        int layer = 0;
        for (size_t lin = 0; lin < c.v.size(); ++lin) {
            if (c.v[lin] != 0.0) {
                std::vector<int> qs(R);
                for (int l = 0; l < R; ++l) qs[l] = -b.q[l] + 2 * idx[l];
                auto it = U.index.find(qs);
                if (it != U.index.end()) {
                    const Block& ub = U.blocks[it->second];
                    int64_t soff = ub.offset;
                    for (int l = 0; l < R; ++l) soff += (int64_t)sz[l].pos.at({b.q[l], qs[l]}) * ub.stride[l];
                    if ((int)layers.size() <= layer) layers.resize(layer + 1);
                    layers[layer++].push_back(
                        make_copy_task(0, soff, 1, b.offset, b.shape, ub.stride, b.stride, c.v[lin] / nrm));
                }
            }
            for (int l = R - 1; l >= 0; --l) {
                if (++idx[l] < c.shape[l]) break;
                idx[l] = 0;
            }
        }
    }
    const bool f64 = U.dtype == SYMTEN_F64;
    std::vector<BufferPtr> keep;
    for (auto& tasks : layers) {
        if (tasks.empty()) continue;
        validate_tasks(tasks, {U.elems, out->elems});
        std::vector<int64_t> prefix;
        copy_prefix(tasks, prefix);
        BufferPtr dt, dp;
        upload_sync(dt, tasks.data(), tasks.size() * sizeof(CopyTask));
        upload_sync(dp, prefix.data(), prefix.size() * sizeof(int64_t));
        copy_launch_arg((const CopyTask*)dt->ptr, (const int64_t*)dp->ptr, (int)tasks.size(), prefix.back(),
                        {U.data(), out->data()}, f64, /*accumulate*/ 4, stream);
        keep.push_back(dt);
        keep.push_back(dp);
    }
    HIPCHK(hipStreamSynchronize(stream));
    return out;
}

// ------------------------------------------------------------ double layer
// a = sum_sigma A A* with the (ket, bra) legs of every bond fused into one
// multiplet leg (Sec. 3.2: rank-4 double-layer tensors).  The fused leg of a
// bond with multiplets {j: n} holds, for every pair (j_ket, j_bra) in
// lexicographic order and every J in j_ket x j_bra, n_ket * n_bra multiplets
// of spin J, row-major in (ket multiplet, bra multiplet).  The fusion map is
// the unitary F[ket, bra, fused] whose blocks are w * c_F with the
// Clebsch-Gordan basis tensor c_F of legs (ket dual, bra dual, fused) and
// w = sqrt((2J+1)/(2j_ket+1)); the bra legs belong to A* and run opposite to
// the ket legs, which is where the conjugate representation enters.
//
// Computed in the S^z basis: the U(1) double layer of A's S^z components, a
// change of basis on each fused leg (a U(1) contraction with F written as a
// charge-diagonal matrix), then the projection onto a's multiplet blocks.
// This runs once per site tensor, not per move.
//
// With `op` (a matrix on the physical S^z states, as for the U(1) double
// layer) and project = false, the result stays a U(1) tensor in the S^z basis
// of the fused multiplets: an operator double layer that is not invariant,
// in the basis of an expanded SU(2) environment (su2_to_u1).
TensorPtr double_layer_su2_impl(const Tensor& A, const double* op, bool project, hipStream_t s) {
    check_device_tensor(A, "double_layer");
    if (A.rank() != 5) fail(SYMTEN_E_INVAL, "double_layer: A must have rank 5 (phys, l, u, r, d)");
    const bool f64 = A.dtype == SYMTEN_F64;
    const int prec = f64 ? SYMTEN_PREC_F64 : SYMTEN_PREC_F32;
    TensorPtr Au = su2_to_u1(A, s);
    TensorPtr au = double_layer(*Au, s, op);
    std::vector<Leg> fused(4);
    std::vector<TensorPtr> W(4);
    for (int x = 0; x < 4; ++x) {
        const Leg& v = A.legs[x + 1];
        // multiplets of the fused leg and the first multiplet of each (j_ket, j_bra) pair
        std::map<int, int> nJ;
        std::map<std::array<int, 3>, int> base;
        for (size_t k = 0; k < v.q.size(); ++k)
            for (size_t b = 0; b < v.q.size(); ++b)
                for (int J = std::abs(v.q[k] - v.q[b]); J <= v.q[k] + v.q[b]; J += 2) {
                    base[{v.q[k], v.q[b], J}] = nJ[J];
                    nJ[J] += v.d[k] * v.d[b];
                }
        Leg F;
        F.dir = v.dir;
        for (auto& kv : nJ) { F.q.push_back(kv.first); F.d.push_back(kv.second); }
        fused[x] = F;
        const SzLeg vs = sz_leg(v), fs = sz_leg(F);
        std::vector<int> ket, bra;
        Leg dl;
        double_layer_states(vs.u1, ket, bra, dl);
        if (dl.q != au->legs[x].q || dl.d != au->legs[x].d) fail(SYMTEN_E_INVAL, "internal: double-layer leg");
        // W[fused U(1) state, S^z state of F] (U(1) tensor, charge diagonal)
        auto w = std::make_shared<Tensor>();
        w->group = SYMTEN_U1;
        w->flux = 0;
        w->dtype = A.dtype;
        Leg rows = dl;
        rows.dir = -v.dir;
        w->legs = {rows, fs.u1};
        w->elems = enumerate_blocks(*w);
        std::vector<double> host((size_t)std::max<int64_t>(w->elems, 1), 0.0);
        std::vector<Leg> flegs(3);
        flegs[0].dir = -v.dir;   // ket dual
        flegs[1].dir = v.dir;    // bra dual (the bra leg of A* runs opposite)
        flegs[2].dir = v.dir;    // fused
        std::vector<int> row_in_sector(ket.size());
        {
            std::map<int, int> cnt;
            int o = 0;
            for (size_t r = 0; r < ket.size(); ++r) {
                const int Q = vs.state_of[ket[r]][2] - vs.state_of[bra[r]][2];
                row_in_sector[r] = cnt[Q]++;
                (void)o;
            }
        }
        for (size_t r = 0; r < ket.size(); ++r) {
            const auto& K = vs.state_of[ket[r]];
            const auto& B = vs.state_of[bra[r]];
            const int Q = K[2] - B[2];
            const int jk = K[0], jb = B[0];
            for (int J = std::abs(jk - jb); J <= jk + jb; J += 2) {
                if (std::abs(Q) > J) continue;
                const DenseT& c = cgc_cached(flegs, {jk, jb, J}, {jk});
                const double val = std::sqrt((J + 1.0) / (jk + 1.0)) *
                                   c.v[((int64_t)((K[2] + jk) / 2) * (jb + 1) + (B[2] + jb) / 2) * (J + 1) + (Q + J) / 2];
                if (val == 0.0) continue;
                const int f = base.at({jk, jb, J}) + K[1] * v.dim_of(jb) + B[1];
                auto it = w->index.find(std::vector<int>{Q, Q});
                if (it == w->index.end()) fail(SYMTEN_E_INVAL, "internal: fusion block");
                const Block& wb = w->blocks[it->second];
                const int col = fs.pos.at({J, Q}) + f;
                host[wb.offset + (int64_t)row_in_sector[r] * wb.stride[0] + (int64_t)col * wb.stride[1]] = val;
            }
        }
        w->buf = device_alloc(std::max<int64_t>(w->elems, 1) * w->esize());
        w->meta_only = false;
        if (f64) {
            HIPCHK(hipMemcpy(w->buf->ptr, host.data(), w->elems * 8, hipMemcpyHostToDevice));
        } else {
            std::vector<float> h32(host.begin(), host.end());
            HIPCHK(hipMemcpy(w->buf->ptr, h32.data(), w->elems * 4, hipMemcpyHostToDevice));
        }
        W[x] = w;
    }
    // change of basis on the four legs (each contraction rotates the leg order)
    TensorPtr cur = au;
    std::vector<std::shared_ptr<ContractPlan>> keep;
    for (int x = 0; x < 4; ++x) {
        const int la = 0, lb = 0;
        auto p = plan_contraction(*cur, *W[x], 1, &la, &lb, nullptr, prec);
        keep.push_back(p);
        cur = run_contraction(*p, *cur, *W[x], s);
    }
    if (!project) {
        HIPCHK(hipStreamSynchronize(s));
        return cur;
    }
    TensorPtr a = u1_to_su2(*cur, fused, s);
    HIPCHK(hipStreamSynchronize(s));
    return a;
}

TensorPtr double_layer_su2(const Tensor& A, hipStream_t s) { return double_layer_su2_impl(A, nullptr, true, s); }

TensorPtr double_layer_su2_sz(const Tensor& A, const double* op, hipStream_t s) {
    return double_layer_su2_impl(A, op, false, s);
}

}  // namespace symten

// ------------------------------------------- leg permutation and reversal
namespace symten {
TensorPtr su2_permute_flip(const Tensor& X, const std::vector<int>& perm, const std::vector<int>& flip,
                           hipStream_t s) {
    if (X.group != SYMTEN_SU2) fail(SYMTEN_E_INVAL, "su2_permute_flip: tensor is not SU(2)");
    const int R = X.rank();
    if ((int)perm.size() != R) fail(SYMTEN_E_INVAL, "su2_permute_flip: bad permutation");
    TensorPtr U = su2_to_u1(X, s);
    // the permuted SU(2) legs, the flipped ones reversed
    std::vector<Leg> legs(R);
    for (int j = 0; j < R; ++j) legs[j] = X.legs[perm[j]];
    std::vector<char> fl(R, 0);
    for (int l : flip) {
        if (l < 0 || l >= R) fail(SYMTEN_E_INVAL, "su2_permute_flip: bad leg");
        fl[l] = 1;
    }
    std::vector<SzLeg> szo(R);             // S^z legs before the reversal (after the permutation)
    for (int j = 0; j < R; ++j) szo[j] = sz_leg(legs[j]);
    for (int j = 0; j < R; ++j)
        if (fl[j]) legs[j].dir = -legs[j].dir;
    // target U(1) tensor: S^z legs of the new SU(2) legs, flux 0
    auto V = std::make_shared<Tensor>();
    V->group = SYMTEN_U1;
    V->flux = 0;
    V->dtype = U->dtype;
    for (int j = 0; j < R; ++j) V->legs.push_back(sz_leg(legs[j]).u1);
    V->elems = enumerate_blocks(*V);
    V->meta_only = false;
    V->buf = device_alloc(std::max<int64_t>(V->elems, 1) * V->esize());
    launch_fill_zero(V->data(), ((std::max<int64_t>(V->elems, 1) * V->esize() + 3) / 4) * 4, s);
    // a reversed leg takes the state (j, a, m) to (j, a, -m) with the phase
    // (-1)^(j-m), which keeps the tensor invariant under the reversed law;
    // the two ends of a bond take the same phase, so networks are unchanged.
    // Inside a charge the states run over spins ascending, then multiplets,
    // and charges m and -m hold the same spins at the same positions.
    std::vector<CopyTask> tasks;
    for (const Block& b0 : U->blocks) {
        Block b = b0;                       // the block seen through the permutation
        for (int j = 0; j < R; ++j) {
            b.q[j] = b0.q[perm[j]];
            b.shape[j] = b0.shape[perm[j]];
            b.stride[j] = b0.stride[perm[j]];
        }
        std::vector<int> key = b.q;
        for (int j = 0; j < R; ++j)
            if (fl[j]) key[j] = -key[j];
        const Block& d = V->blocks[V->index.at(key)];
        // ranges of the reversed legs: one per spin present in the charge
        struct Rg { int start, len, sign; };
        std::vector<std::vector<Rg>> rg(R);
        for (int j = 0; j < R; ++j) {
            if (!fl[j]) { rg[j].push_back({0, b.shape[j], 1}); continue; }
            const int m = b.q[j];
            for (size_t i = 0; i < legs[j].q.size(); ++i) {
                const int t = legs[j].q[i];
                if (t < std::abs(m) || (t - m) % 2 != 0) continue;
                const int sign = (((t - m) / 2) % 2 == 0) ? 1 : -1;
                rg[j].push_back({szo[j].pos.at({t, m}), legs[j].d[i], sign});
            }
        }
        std::vector<size_t> it(R, 0);
        while (true) {
            std::vector<int> dims(R);
            int64_t so = b.offset, dof = d.offset;
            int sign = 1;
            for (int j = 0; j < R; ++j) {
                const Rg& r = rg[j][it[j]];
                dims[j] = r.len;
                so += (int64_t)r.start * b.stride[j];
                dof += (int64_t)r.start * d.stride[j];
                sign *= r.sign;
            }
            std::vector<int64_t> ss(b.stride.begin(), b.stride.end()), ds(d.stride.begin(), d.stride.end());
            tasks.push_back(make_copy_task(0, so, 1, dof, dims, ss, ds, (double)sign));
            int j = R - 1;
            while (j >= 0 && ++it[j] == rg[j].size()) it[j--] = 0;
            if (j < 0) break;
        }
    }
    if (!tasks.empty()) {
        validate_tasks(tasks, {U->elems, V->elems});
        std::vector<int64_t> prefix;
        copy_prefix(tasks, prefix);
        BufferPtr dt, dp;
        upload_sync(dt, tasks.data(), tasks.size() * sizeof(CopyTask));
        upload_sync(dp, prefix.data(), prefix.size() * sizeof(int64_t));
        const bool f64 = U->dtype == SYMTEN_F64;
        copy_launch_arg((const CopyTask*)dt->ptr, (const int64_t*)dp->ptr, (int)tasks.size(), prefix.back(),
                        {U->data(), V->data()}, f64, f64 ? 1 : 0, s);
        HIPCHK(hipStreamSynchronize(s));
    }
    return u1_to_su2(*V, legs, s);
}

TensorPtr su2_sign_half_integer(const Tensor& X, int leg, hipStream_t s) {
    if (X.group != SYMTEN_SU2) fail(SYMTEN_E_INVAL, "su2_sign_half_integer: tensor is not SU(2)");
    auto out = std::make_shared<Tensor>(X);
    out->meta_only = false;
    out->buf = device_alloc(std::max<int64_t>(X.elems, 1) * X.esize());
    std::vector<CopyTask> tasks;
    for (size_t i = 0; i < X.blocks.size(); ++i) {
        const Block& b = X.blocks[i];
        std::vector<int64_t> st(b.stride.begin(), b.stride.end());
        tasks.push_back(make_copy_task(0, b.offset, 1, b.offset, b.shape, st, st, (b.q[leg] % 2) ? -1.0 : 1.0));
    }
    if (!tasks.empty()) {
        validate_tasks(tasks, {X.elems, X.elems});
        std::vector<int64_t> prefix;
        copy_prefix(tasks, prefix);
        BufferPtr dt, dp;
        upload_sync(dt, tasks.data(), tasks.size() * sizeof(CopyTask));
        upload_sync(dp, prefix.data(), prefix.size() * sizeof(int64_t));
        const bool f64 = X.dtype == SYMTEN_F64;
        copy_launch_arg((const CopyTask*)dt->ptr, (const int64_t*)dp->ptr, (int)tasks.size(), prefix.back(),
                        {X.data(), out->data()}, f64, f64 ? 1 : 0, s);
        HIPCHK(hipStreamSynchronize(s));
    }
    return out;
}
}  // namespace symten
