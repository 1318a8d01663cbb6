// Sector matching on the device (Sec. 2: a contraction pairs the blocks
// whose labels agree on the contracted legs, and the products are grouped by
// the labels of the open legs).
//
// One workgroup enumerates, from the leg tables alone (sector labels, dims
// and directions of every leg, the flux, the charge modulus):
//   1. the allowed blocks of A and of B (sum of dir * q equal to the flux),
//      in canonical order: label tuples lexicographic, leg 0 slowest;
//   2. the matched pairs (i, j) of an A block and a B block with equal labels
//      on the contracted legs, in lexicographic (i, j) order, with their
//      useful flops 2 m n k;
//   3. the output blocks reached by at least one pair (A's open labels, then
//      B's open labels, lexicographic), and for each pair its output block.
// Every list is written by a block-wide prefix sum over flags, so the order
// is deterministic.  Lists longer than the caller's capacities are cut, and
// the full counts are reported with a status flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace symten {

namespace {
constexpr int kMatchThreads = 1024;
constexpr int kMaxLegSectors = 64;

struct MatchArgs {
    int ra, rb, ncon, modulus;
    int flux_a, flux_b;
    int nsec_a[kMaxCopyRank], nsec_b[kMaxCopyRank];
    int dir_a[kMaxCopyRank], dir_b[kMaxCopyRank];
    int con_a[kMaxCopyRank], con_b[kMaxCopyRank];     // contracted legs, in pairs
    int free_a[kMaxCopyRank], free_b[kMaxCopyRank];
    int nfree_a, nfree_b;
    const int* lab_a;   // [ra][kMaxLegSectors] labels, ascending per leg
    const int* dim_a;
    const int* lab_b;
    const int* dim_b;
    int64_t space_a, space_b, space_out;   // sizes of the label-tuple spaces
    int64_t cap_blocks, pair_cap, out_cap;
    int* blocks_a;          // [cap_blocks] tuple index of each allowed A block
    int* blocks_b;
    int* out_flag;          // [space_out] scratch: 1 where an output is reached
    int* out_pos;           // [space_out] scratch: its output block index
    symten_pair* pairs;     // [pair_cap]
    int* out_labels;        // [out_cap][nfree_a + nfree_b]
    int64_t* counts;        // [5]: A blocks, B blocks, pairs, output blocks, status
};

// Exclusive prefix sum of one int per thread over the workgroup; returns the
// thread's offset and writes the total to *total.
__device__ int block_exclusive_scan(int v, int* total) {
    __shared__ int wsum[kMatchThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < kMatchThreads / 64; ++w) {
            const int t = wsum[w];
            wsum[w] = acc;
            acc += t;
        }
        *total = acc;
    }
    __syncthreads();
    const int r = wsum[wave] + x - v;
    __syncthreads();
    return r;
}

__device__ int norm_charge(long q, int m) { return m ? (int)(((q % m) + m) % m) : (int)q; }

// Label-tuple index t of a tensor with `rank` legs -> sector index per leg
// (leg 0 slowest).
__device__ void decode(int64_t t, int rank, const int* nsec, int* s) {
    for (int l = rank - 1; l >= 0; --l) {
        s[l] = (int)(t % nsec[l]);
        t /= nsec[l];
    }
}

// Allowed blocks of one tensor: tuple indices in lexicographic order.
__device__ int64_t enumerate(int64_t space, int rank, const int* nsec, const int* dir, const int* lab, int flux,
                             int modulus, int* out, int64_t cap) {
    __shared__ int tot;
    int64_t base = 0;
    for (int64_t c0 = 0; c0 < space; c0 += kMatchThreads) {
        const int64_t t = c0 + threadIdx.x;
        int ok = 0;
        if (t < space) {
            int s[kMaxCopyRank];
            decode(t, rank, nsec, s);
            long q = 0;
            for (int l = 0; l < rank; ++l) q += (long)dir[l] * lab[l * kMaxLegSectors + s[l]];
            ok = norm_charge(q - flux, modulus) == 0;
        }
        const int p = block_exclusive_scan(ok, &tot);
        if (ok && base + p < cap) out[base + p] = (int)t;
        base += tot;
    }
    return base;
}

__global__ __launch_bounds__(kMatchThreads) void match_kernel(MatchArgs a) {
    __shared__ int tot;
    const int64_t na = enumerate(a.space_a, a.ra, a.nsec_a, a.dir_a, a.lab_a, a.flux_a, a.modulus, a.blocks_a,
                                 a.cap_blocks);
    const int64_t nb = enumerate(a.space_b, a.rb, a.nsec_b, a.dir_b, a.lab_b, a.flux_b, a.modulus, a.blocks_b,
                                 a.cap_blocks);
    const bool blocks_ok = na <= a.cap_blocks && nb <= a.cap_blocks;
    for (int64_t i = threadIdx.x; i < a.space_out; i += kMatchThreads) a.out_flag[i] = 0;
    __syncthreads();
    int64_t npairs = 0;
    if (blocks_ok) {
        // matched pairs in (i, j) order; mark the output tuple of each
        const int64_t space = na * nb;
        for (int64_t c0 = 0; c0 < space; c0 += kMatchThreads) {
            const int64_t t = c0 + threadIdx.x;
            int ok = 0;
            int sa[kMaxCopyRank], sb[kMaxCopyRank];
            int64_t flops = 0, oidx = 0;
            if (t < space) {
                decode(a.blocks_a[t / nb], a.ra, a.nsec_a, sa);
                decode(a.blocks_b[t % nb], a.rb, a.nsec_b, sb);
                ok = 1;
                int64_t k = 1;
                for (int c = 0; c < a.ncon; ++c) {
                    const int la = a.lab_a[a.con_a[c] * kMaxLegSectors + sa[a.con_a[c]]];
                    const int lb = a.lab_b[a.con_b[c] * kMaxLegSectors + sb[a.con_b[c]]];
                    if (la != lb) ok = 0;
                    k *= a.dim_a[a.con_a[c] * kMaxLegSectors + sa[a.con_a[c]]];
                }
                int64_t m = 1, n = 1;
                for (int f = 0; f < a.nfree_a; ++f) {
                    const int l = a.free_a[f];
                    m *= a.dim_a[l * kMaxLegSectors + sa[l]];
                    oidx = oidx * a.nsec_a[l] + sa[l];
                }
                for (int f = 0; f < a.nfree_b; ++f) {
                    const int l = a.free_b[f];
                    n *= a.dim_b[l * kMaxLegSectors + sb[l]];
                    oidx = oidx * a.nsec_b[l] + sb[l];
                }
                flops = 2 * m * n * k;
            }
            const int p = block_exclusive_scan(ok, &tot);
            if (ok) {
                a.out_flag[oidx] = 1;
                if (npairs + p < a.pair_cap) {
                    symten_pair& q = a.pairs[npairs + p];
                    q.a_block = (int32_t)(t / nb);
                    q.b_block = (int32_t)(t % nb);
                    q.out_block = (int32_t)oidx;   // tuple index for now
                    q.flops = flops;
                }
            }
            npairs += tot;
        }
    }
    __syncthreads();
    // output blocks: reached tuples in lexicographic order
    int64_t nout = 0;
    const int ro = a.nfree_a + a.nfree_b;
    for (int64_t c0 = 0; c0 < a.space_out; c0 += kMatchThreads) {
        const int64_t t = c0 + threadIdx.x;
        const int ok = t < a.space_out ? a.out_flag[t] : 0;
        const int p = block_exclusive_scan(ok, &tot);
        if (ok) {
            a.out_pos[t] = (int)(nout + p);
            if (nout + p < a.out_cap) {
                int64_t r = t;
                for (int f = ro - 1; f >= 0; --f) {
                    const bool fa = f < a.nfree_a;
                    const int l = fa ? a.free_a[f] : a.free_b[f - a.nfree_a];
                    const int ns = fa ? a.nsec_a[l] : a.nsec_b[l];
                    const int s = (int)(r % ns);
                    r /= ns;
                    a.out_labels[(nout + p) * ro + f] = fa ? a.lab_a[l * kMaxLegSectors + s] : a.lab_b[l * kMaxLegSectors + s];
                }
            }
        }
        nout += tot;
    }
    __syncthreads();
    const int64_t stored = npairs < a.pair_cap ? npairs : a.pair_cap;
    for (int64_t i = threadIdx.x; i < stored; i += kMatchThreads)
        a.pairs[i].out_block = a.out_pos[a.pairs[i].out_block];
    if (threadIdx.x == 0) {
        a.counts[0] = na;
        a.counts[1] = nb;
        a.counts[2] = npairs;
        a.counts[3] = nout;
        a.counts[4] = (!blocks_ok || npairs > a.pair_cap || nout > a.out_cap) ? 1 : 0;
    }
}
}  // namespace

void match_blocks(const Tensor& A, const Tensor& B, int ncon, const int* legsA, const int* legsB,
                  symten_pair* pairs, int64_t pair_cap, int* out_labels, int64_t out_cap, int64_t* counts,
                  hipStream_t s) {
    if (A.group != B.group || !abelian(A.group)) fail(SYMTEN_E_UNSUPPORTED, "match_blocks: U(1) or Z2 tensors");
    const int ra = A.rank(), rb = B.rank();
    if (ncon < 0 || ncon > ra || ncon > rb || (ncon > 0 && (!legsA || !legsB)))
        fail(SYMTEN_E_INVAL, "match_blocks: bad contracted legs");
    if (!counts || (pair_cap > 0 && !pairs) || (out_cap > 0 && !out_labels) || pair_cap < 0 || out_cap < 0)
        fail(SYMTEN_E_INVAL, "match_blocks: null output or negative capacity");
    MatchArgs m{};
    m.ra = ra;
    m.rb = rb;
    m.ncon = ncon;
    m.modulus = charge_mod(A.group);
    m.flux_a = A.flux;
    m.flux_b = B.flux;
    std::vector<int> used_a(ra, 0), used_b(rb, 0);
    for (int c = 0; c < ncon; ++c) {
        if (legsA[c] < 0 || legsA[c] >= ra || legsB[c] < 0 || legsB[c] >= rb || used_a[legsA[c]]++ ||
            used_b[legsB[c]]++)
            fail(SYMTEN_E_INVAL, "match_blocks: leg index out of range or repeated");
        if (A.legs[legsA[c]].dir != -B.legs[legsB[c]].dir || !A.legs[legsA[c]].same_sectors(B.legs[legsB[c]]))
            fail(SYMTEN_E_LEGS, "match_blocks: contracted legs must be dual");
        m.con_a[c] = legsA[c];
        m.con_b[c] = legsB[c];
    }
    std::vector<int> tab(4 * kMaxCopyRank * kMaxLegSectors, 0);
    int64_t space_out = 1;
    auto fill = [&](const Tensor& X, int* nsec, int* dir, int* lab, int* dim, int64_t& space) {
        space = 1;
        for (int l = 0; l < X.rank(); ++l) {
            const Leg& L = X.legs[l];
            if ((int)L.q.size() > kMaxLegSectors) fail(SYMTEN_E_CAPACITY, "match_blocks: more than 64 sectors on a leg");
            nsec[l] = (int)L.q.size();
            dir[l] = L.dir;
            for (int q = 0; q < nsec[l]; ++q) {
                lab[l * kMaxLegSectors + q] = L.q[q];
                dim[l * kMaxLegSectors + q] = L.d[q];
            }
            space *= std::max(1, nsec[l]);
            if (nsec[l] == 0) space = 0;
        }
    };
    const int stride = kMaxCopyRank * kMaxLegSectors;
    fill(A, m.nsec_a, m.dir_a, tab.data(), tab.data() + stride, m.space_a);
    fill(B, m.nsec_b, m.dir_b, tab.data() + 2 * stride, tab.data() + 3 * stride, m.space_b);
    for (int l = 0; l < ra; ++l)
        if (!used_a[l]) { m.free_a[m.nfree_a++] = l; space_out *= std::max(1, m.nsec_a[l]); }
    for (int l = 0; l < rb; ++l)
        if (!used_b[l]) { m.free_b[m.nfree_b++] = l; space_out *= std::max(1, m.nsec_b[l]); }
    if (m.nfree_a + m.nfree_b == 0) fail(SYMTEN_E_UNSUPPORTED, "match_blocks: full contraction to a scalar");
    if (m.space_a > (1LL << 30) || m.space_b > (1LL << 30) || space_out > (1LL << 26))
        fail(SYMTEN_E_CAPACITY, "match_blocks: label-tuple space too large");
    m.space_out = space_out;
    m.cap_blocks = std::max<int64_t>(A.blocks.size(), B.blocks.size());   // exact block counts (host enumeration)
    m.pair_cap = pair_cap;
    m.out_cap = out_cap;
    m.pairs = pairs;
    m.out_labels = out_labels;
    m.counts = counts;
    // device work buffers (stream-ordered pool): leg tables, block lists, output flags
    const int64_t nb_tab = (int64_t)tab.size() * sizeof(int);
    BufferPtr w = device_alloc(nb_tab + 2 * 4 * m.cap_blocks + 2 * 4 * space_out + 64);
    char* p = (char*)w->ptr;
    HIPCHK(hipMemcpyAsync(p, tab.data(), nb_tab, hipMemcpyHostToDevice, s));
    m.lab_a = (const int*)p;
    m.dim_a = (const int*)p + stride;
    m.lab_b = (const int*)p + 2 * stride;
    m.dim_b = (const int*)p + 3 * stride;
    m.blocks_a = (int*)(p + nb_tab);
    m.blocks_b = m.blocks_a + m.cap_blocks;
    m.out_flag = m.blocks_b + m.cap_blocks;
    m.out_pos = m.out_flag + space_out;
    hipLaunchKernelGGL(match_kernel, dim3(1), dim3(kMatchThreads), 0, s, m);
    HIPCHK(hipGetLastError());
}

}  // namespace symten
