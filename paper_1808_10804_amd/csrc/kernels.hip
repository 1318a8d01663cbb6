// Device kernels of libsymten for gfx950 (CDNA4, 64-wide wavefronts).
//
//  * copy_kernel      strided gather of tensor blocks into GEMM panels
//                     (block -> [open, contracted] layout, K-concatenated per
//                     charge sector), with type conversion and zero fill.
//  * gemm_kernel      grouped GEMM C_g = A_g B_g^T over all charge sectors of
//                     one or many contractions: LDS-staged tiles, MFMA
//                     f64 16x16x4, f32 32x32x2, bf16 32x32x16 (plain and
//                     three-product split precision), FP32/FP64 accumulation.
//  * double_layer     a = sum_s A A* with fused (ket, bra) legs.
//  * reductions       FP64 sum of squares (deterministic two-pass), scaling,
//                     casts, sign gauge of projector rows.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <cstdio>
#include <vector>
#include <mutex>
#include <algorithm>

#include "internal.hpp"

namespace symten {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f16_t __attribute__((ext_vector_type(16)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned short us8_t __attribute__((ext_vector_type(8)));

// Pointer table passed by value (single contraction) or by device pointer
// (batched launches prepared ahead of time).
struct ArgPtrs {
    void* p[16];
    __device__ __forceinline__ void* get(int i) const { return p[i]; }
};
struct DevPtrs {
    void* const* p;
    __device__ __forceinline__ void* get(int i) const { return p[i]; }
};

// ===================================================================== copy
constexpr int kCopyChunk = 1024;
constexpr int kCopyThreads = 256;

__device__ __forceinline__ unsigned short f32_to_bf16_rn(float x) {
    // round to nearest, ties to even, on the bit pattern (finite inputs;
    // NaN keeps a quiet mantissa bit)
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
    return __uint_as_float(((uint32_t)h) << 16);
}

// Destination kinds of the gather: float, double, one bf16 plane, the
// split x = hi + lo with hi = bf16(x), lo = bf16(x - hi) in two planes,
// accumulation (dst += scale * src) in the source type, or the split
// x = hi + mid + lo with mid = bf16(x - hi), lo = bf16(x - hi - mid) in three
// planes (each plane lo_off elements after the previous one).
enum : int { kDstF32 = 0, kDstF64 = 1, kDstBF16 = 2, kDstSplit = 3, kDstAcc = 4, kDstSplit3 = 5 };

// x as PL bf16 planes: plane 0 = bf16(x); with two planes plane 1 =
// bf16(x - plane 0); with three, plane 1 = bf16(x - plane 0) and plane 2 =
// bf16(x - plane 0 - plane 1) (the differences are exact in FP32).  The
// gather's split destinations store the same values.
template <int PL>
__device__ __forceinline__ void bf16_planes(float x, unsigned short* h) {
    h[0] = f32_to_bf16_rn(x);
    if constexpr (PL >= 2) {
        const float r1 = x - bf16_to_f32(h[0]);
        h[1] = f32_to_bf16_rn(r1);
        if constexpr (PL == 3) h[2] = f32_to_bf16_rn(r1 - bf16_to_f32(h[1]));
    }
}

// One destination element of the gather: conversion to the destination kind.
template <typename TS, int DK, typename AT>
__device__ __forceinline__ void copy_store(void* dstv, int64_t dofs, int64_t lo_off, AT sv, bool have_src) {
    if constexpr (DK == kDstAcc) {
        if (have_src) ((TS*)dstv)[dofs] += (TS)sv;
    } else if constexpr (DK == kDstF64) {
        ((double*)dstv)[dofs] = (double)sv;
    } else if constexpr (DK == kDstF32) {
        ((float*)dstv)[dofs] = (float)sv;
    } else {
        const float v = (float)sv;
        const unsigned short h = f32_to_bf16_rn(v);
        ((unsigned short*)dstv)[dofs] = h;
        if constexpr (DK == kDstSplit) ((unsigned short*)dstv)[dofs + lo_off] = f32_to_bf16_rn(v - bf16_to_f32(h));
        if constexpr (DK == kDstSplit3) {
            // both differences are exact in FP32: hi and mid take the leading
            // 8 + 8 significand bits of v
            const float r1 = v - bf16_to_f32(h);
            const unsigned short m = f32_to_bf16_rn(r1);
            ((unsigned short*)dstv)[dofs + lo_off] = m;
            ((unsigned short*)dstv)[dofs + 2 * lo_off] = f32_to_bf16_rn(r1 - bf16_to_f32(m));
        }
    }
}

// Strided gather over a task list.  A task's elements are cut into chunks:
// 1024 consecutive elements of a direct copy, or one tile of a transposing
// copy (read along the source's unit-stride dim into LDS, written along the
// destination's unit-stride dim).  Each workgroup takes one piece, up to
// kCopyGroup consecutive chunks of one task: it finds the task by bisection
// over the pieces' prefix sums, decodes it once and issues the loads of all
// its chunks before the first store.  A task may sum several equally strided
// sources with their scalars (SU(2) tree-sibling blocks).
constexpr int kCopyRun = kCopyChunk / kCopyThreads;   // elements per thread and chunk
constexpr int kTileLds = kCopyChunk + 64;              // LDS elements of one tile

template <typename TS, int DK, typename AT, typename G>
__device__ __forceinline__ void copy_tiles(const CopyTask& T, int64_t first, int ng, void* dstv, AT* tile,
                                           G gather) {
    // TO destination-contiguous x TI source-contiguous elements per tile
    const int rank = T.rank;
    const int din = T.tr_in, dout = T.tr_out;
    const int lgo = T.lg_out, lgi = 10 - T.lg_out;
    const int TO = 1 << lgo, TI = 1 << lgi;
    const int LS = TI + 1;   // LDS row stride
    const int Din = T.dims[din], Dout = T.dims[dout];
    const int nto = (Dout + TO - 1) >> lgo, nti = (Din + TI - 1) >> lgi;
    const int64_t ssi = T.sstride[din], sso = T.sstride[dout];
    const int64_t dsi = T.dstride[din], dso = T.dstride[dout];
    int64_t dbase[kCopyGroup];
    int ib[kCopyGroup], ob[kCopyGroup];
    AT v[kCopyGroup][kCopyRun];
    // loads of every tile of the piece
#pragma unroll
    for (int j = 0; j < kCopyGroup; ++j) {
        if (j >= ng) break;
        int64_t r = first + j;
        const int to = (int)(r % nto);
        r /= nto;
        const int ti = (int)(r % nti);
        r /= nti;
        int64_t so = T.src_off, dofs = T.dst_off;
        for (int k = rank - 1; k >= 0; --k) {
            if (k == din || k == dout) continue;
            const int ik = (int)(r % T.dims[k]);
            r /= T.dims[k];
            so += (int64_t)ik * T.sstride[k];
            dofs += (int64_t)ik * T.dstride[k];
        }
        dbase[j] = dofs;
        ib[j] = ti << lgi;
        ob[j] = to << lgo;
#pragma unroll
        for (int q = 0; q < kCopyRun; ++q) {
            const int e = threadIdx.x + q * kCopyThreads;
            const int gi = ib[j] + (e & (TI - 1)), go = ob[j] + (e >> lgi);
            if (gi < Din && go < Dout) v[j][q] = gather(so + gi * ssi + go * sso);
        }
    }
#pragma unroll
    for (int j = 0; j < kCopyGroup; ++j) {
        if (j >= ng) break;
#pragma unroll
        for (int q = 0; q < kCopyRun; ++q) {
            const int e = threadIdx.x + q * kCopyThreads;
            const int ii = e & (TI - 1), oo = e >> lgi;
            if (ib[j] + ii < Din && ob[j] + oo < Dout) tile[j * kTileLds + oo * LS + ii] = v[j][q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kCopyGroup; ++j) {
        if (j >= ng) break;
#pragma unroll
        for (int q = 0; q < kCopyRun; ++q) {
            const int e = threadIdx.x + q * kCopyThreads;
            const int oo = e & (TO - 1), ii = e >> lgo;
            const int gi = ib[j] + ii, go = ob[j] + oo;
            if (gi < Din && go < Dout)
                copy_store<TS, DK>(dstv, dbase[j] + gi * dsi + go * dso, T.lo_off,
                                   tile[j * kTileLds + oo * LS + ii], true);
        }
    }
}

template <typename TS, int DK, typename AT, typename G>
__device__ __forceinline__ void copy_runs(const CopyTask& T, int64_t first, int ng, bool have_src, void* dstv,
                                          G gather) {
    // per chunk, each thread copies kCopyRun consecutive elements: the
    // multi-index is decomposed for the first and advanced along the
    // innermost dim
    const int last = T.rank - 1;
    const int dl = T.dims[last];
    const int64_t sl = T.sstride[last], dls = T.dstride[last];
    AT v[kCopyGroup][kCopyRun];
    int64_t dd[kCopyGroup][kCopyRun];
    int n[kCopyGroup];
#pragma unroll
    for (int j = 0; j < kCopyGroup; ++j) {
        n[j] = 0;
        if (j >= ng) continue;
        const int64_t idx0 = (first + j) * kCopyChunk + (int64_t)threadIdx.x * kCopyRun;
        if (idx0 >= T.count) continue;
        n[j] = (int)min<int64_t>(kCopyRun, T.count - idx0);
        int inner = 0;
        int64_t so = 0, dofs = 0;
        auto locate = [&](int64_t idx) {
            uint32_t r = (uint32_t)idx;
            so = T.src_off;
            dofs = T.dst_off;
            for (int k = last; k >= 0; --k) {
                const uint32_t dk = (uint32_t)T.dims[k];
                const uint32_t q = r / dk;
                const uint32_t ik = r - q * dk;
                if (k == last) inner = (int)ik;
                r = q;
                so += (int64_t)ik * T.sstride[k];
                dofs += (int64_t)ik * T.dstride[k];
            }
        };
        locate(idx0);
#pragma unroll
        for (int u = 0; u < kCopyRun; ++u) {
            if (u >= n[j]) break;
            dd[j][u] = dofs;
            v[j][u] = have_src ? gather(so) : (AT)0;
            if (++inner < dl) {
                so += sl;
                dofs += dls;
            } else if (u + 1 < n[j]) {
                locate(idx0 + u + 1);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kCopyGroup; ++j) {
        if constexpr (DK == kDstBF16 || DK == kDstSplit || DK == kDstSplit3) {
            // four consecutive, aligned destinations: one vector per plane
            constexpr int PL = DK == kDstBF16 ? 1 : (DK == kDstSplit ? 2 : 3);
            if (n[j] == kCopyRun && (dd[j][0] & 3) == 0 && dd[j][1] == dd[j][0] + 1 && dd[j][2] == dd[j][0] + 2 &&
                dd[j][3] == dd[j][0] + 3) {
                unsigned short h[kCopyRun][3];
#pragma unroll
                for (int u = 0; u < kCopyRun; ++u) bf16_planes<PL>((float)v[j][u], h[u]);
#pragma unroll
                for (int p = 0; p < PL; ++p) {
                    const uint2 w = {(uint32_t)h[0][p] | ((uint32_t)h[1][p] << 16),
                                     (uint32_t)h[2][p] | ((uint32_t)h[3][p] << 16)};
                    *(uint2*)((unsigned short*)dstv + dd[j][0] + p * T.lo_off) = w;
                }
                continue;
            }
        }
#pragma unroll
        for (int u = 0; u < kCopyRun; ++u)
            if (u < n[j]) copy_store<TS, DK>(dstv, dd[j][u], T.lo_off, v[j][u], have_src);
    }
}

template <class Ptrs, typename TS, int DK>
__global__ __launch_bounds__(kCopyThreads) void copy_kernel(const CopyTask* __restrict__ tasks,
                                                            const int64_t* __restrict__ piece_prefix,
                                                            int ntasks, Ptrs ptrs) {
    using AT = std::conditional_t<DK == kDstF64, double, TS>;   // arithmetic type
    __shared__ AT tile[kCopyGroup * kTileLds];
    const int64_t w = blockIdx.x;
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {                       // last task with prefix <= w
        int mid = (lo + hi + 1) >> 1;
        if (piece_prefix[mid] <= w) lo = mid; else hi = mid - 1;
    }
    const CopyTask& T = tasks[lo];
    const int64_t first = (w - piece_prefix[lo]) * kCopyGroup;
    const int ng = (int)min<int64_t>(kCopyGroup, (int64_t)T.nchunks - first);
    const TS* __restrict__ src = T.src_buf >= 0 ? (const TS*)ptrs.get(T.src_buf) : nullptr;
    void* dstv = ptrs.get(T.dst_buf);
    const double scale = T.scale;
    auto gather = [&](int64_t so) -> AT {
        AT sv = (AT)src[so] * (AT)scale;
        const int64_t rel = so - T.src_off;
        for (int t = 0; t < T.nextra; ++t) sv += (AT)src[T.xsrc_off[t] + rel] * (AT)T.xscale[t];
        return sv;
    };
    if (T.tr_in >= 0)
        copy_tiles<TS, DK, AT>(T, first, ng, dstv, tile, gather);
    else
        copy_runs<TS, DK, AT>(T, first, ng, src != nullptr, dstv, gather);
}

// ===================================================================== gemm
// Tile configurations.  256 threads = 4 waves in a 2x2 grid; each wave
// owns a (BM/2) x (BN/2) sub-tile made of MT x MT MFMA tiles.
template <int BM_, int BN_, int BK_>
struct TileShape {
    static constexpr int BM = BM_, BN = BN_, BK = BK_;
};

// ---- FP64: v_mfma_f64_16x16x4f64 -----------------------------------------
// lane l: A[row l%16][k l/16], B[col l%16][k l/16]; acc e: row l/16 + 4*e, col l%16 (checked on gfx950)
template <class Ptrs, class S>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const TileWork* __restrict__ tiles, int ntiles,
                                                       int* __restrict__ queue,
                                                       const GemmGroup* __restrict__ groups,
                                                       Ptrs ptrs, double* __restrict__ ws) {
    constexpr int BM = S::BM, BN = S::BN, BK = S::BK;
    constexpr int LDK = BK + 1;
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TI = WM / 16, TJ = WN / 16;
    __shared__ double As[BM * LDK];
    __shared__ double Bs[BN * LDK];

  // Entry t of the list belongs to XCD t mod 8, and workgroup b runs on XCD
  // b mod 8.  Each workgroup starts with its own entry; with a queue (a
  // persistent grid smaller than the list), it then takes the next free row
  // of its XCD's list from that XCD's counter.
  __shared__ int next_row;
  for (int t = blockIdx.x; t < ntiles;) {
    const TileWork tw = tiles[t];
    if (tw.group >= 0) {   // group < 0: padding of the per-XCD lists
    const GemmGroup g = groups[tw.group];
    const double* __restrict__ A = (const double*)ptrs.get(g.a_buf) + g.a_off;
    const double* __restrict__ B = (const double*)ptrs.get(g.b_buf) + g.b_off;
    double* __restrict__ C = (double*)ptrs.get(g.c_buf) + g.c_off;
    const int m0 = tw.tm * BM, n0 = tw.tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

    constexpr int VA = BM * BK / 2 / 256;   // double2 per thread for A
    constexpr int VB = BN * BK / 2 / 256;
    static_assert(VA >= 1 && VB >= 1, "tile too small");
    double2 ra[VA], rb[VB];

    auto gload = [&](int k0) {
#pragma unroll
        for (int v = 0; v < VA; ++v) {
            const int idx = tid + v * 256;
            const int r = idx / (BK / 2), kq = (idx % (BK / 2)) * 2;
            const int gr = m0 + r, gk = k0 + kq;
            ra[v] = (gr < g.M && gk < g.lda) ? *(const double2*)(A + (int64_t)gr * g.lda + gk)
                                             : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int v = 0; v < VB; ++v) {
            const int idx = tid + v * 256;
            const int r = idx / (BK / 2), kq = (idx % (BK / 2)) * 2;
            const int gr = n0 + r, gk = k0 + kq;
            rb[v] = (gr < g.N && gk < g.ldb) ? *(const double2*)(B + (int64_t)gr * g.ldb + gk)
                                             : make_double2(0.0, 0.0);
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int v = 0; v < VA; ++v) {
            const int idx = tid + v * 256;
            const int r = idx / (BK / 2), kq = (idx % (BK / 2)) * 2;
            As[r * LDK + kq] = ra[v].x;
            As[r * LDK + kq + 1] = ra[v].y;
        }
#pragma unroll
        for (int v = 0; v < VB; ++v) {
            const int idx = tid + v * 256;
            const int r = idx / (BK / 2), kq = (idx % (BK / 2)) * 2;
            Bs[r * LDK + kq] = rb[v].x;
            Bs[r * LDK + kq + 1] = rb[v].y;
        }
    };

    d4_t acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    const int kb = tw.k0, ke = tw.k1;   // this item's K range (whole stages but the last)
    if (ke > kb) gload(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        sstore();
        __syncthreads();
        if (k0 + BK < ke) gload(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double a[TI], b[TJ];
#pragma unroll
            for (int i = 0; i < TI; ++i) a[i] = As[(wm + i * 16 + (lane & 15)) * LDK + kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < TJ; ++j) b[j] = Bs[(wn + j * 16 + (lane & 15)) * LDK + kk + (lane >> 4)];
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // a whole-K item writes C; a split-K part writes its partial tile
    double* __restrict__ W = ws + (int64_t)(tw.slot < 0 ? 0 : tw.slot) * BM * BN;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int col = n0 + wn + j * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm + i * 16 + (lane >> 4) + 4 * e;
                if (tw.slot >= 0) W[(row - m0) * BN + (col - n0)] = acc[i][j][e];
                else if (row < g.M && col < g.N) C[(int64_t)row * g.ldc + col] = acc[i][j][e];
            }
        }
    }
    if (!queue) break;
    if (threadIdx.x == 0) next_row = (int)(gridDim.x >> 3) + atomicAdd(&queue[blockIdx.x & 7], 1);
    __syncthreads();
    t = next_row * 8 + (int)(blockIdx.x & 7);
    __syncthreads();
  }
}

// ---- FP32: v_mfma_f32_32x32x2f32 -------------------------------------------
// f32 32x32x2: lane l: A[row l%32][k l/32]; bf16 32x32x16: A[row l%32][k 8*(l/32)+0..7]
// acc i (16 values): row 8*(i/4) + 4*(l/32) + i%4, col l%32
// One LDS stage with the next K stage prefetched into registers during the
// MFMAs (two LDS stages, one barrier each, measured slower: the doubled LDS
// lowers occupancy).
template <class Ptrs, class S>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const TileWork* __restrict__ tiles, int ntiles,
                                                       int* __restrict__ queue,
                                                       const GemmGroup* __restrict__ groups,
                                                       Ptrs ptrs, float* __restrict__ ws) {
    constexpr int BM = S::BM, BN = S::BN, BK = S::BK;
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TI = WM / 32, TJ = WN / 32;
    static_assert(TI >= 1 && TJ >= 1, "tile too small");
    constexpr int LDF = BK + 1;   // LDS row stride in floats
    __shared__ float As[BM * LDF];
    __shared__ float Bs[BN * LDF];

  // Entry t of the list belongs to XCD t mod 8, and workgroup b runs on XCD
  // b mod 8.  Each workgroup starts with its own entry; with a queue (a
  // persistent grid smaller than the list), it then takes the next free row
  // of its XCD's list from that XCD's counter.
  __shared__ int next_row;
  for (int t = blockIdx.x; t < ntiles;) {
    const TileWork tw = tiles[t];
    if (tw.group >= 0) {   // group < 0: padding of the per-XCD lists
    const GemmGroup g = groups[tw.group];
    const float* __restrict__ A = (const float*)ptrs.get(g.a_buf) + g.a_off;
    const float* __restrict__ B = (const float*)ptrs.get(g.b_buf) + g.b_off;
    float* __restrict__ C = (float*)ptrs.get(g.c_buf) + g.c_off;
    const int m0 = tw.tm * BM, n0 = tw.tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

    constexpr int VA = BM * BK / 4 / 256;   // float4 per thread
    constexpr int VB = BN * BK / 4 / 256;
    static_assert(VA >= 1 && VB >= 1, "tile too small");
    float4 ra[VA], rb[VB];

    auto gload = [&](int k0) {
#pragma unroll
        for (int v = 0; v < VA; ++v) {
            const int idx = tid + v * 256;
            const int r = idx / (BK / 4), kq = (idx % (BK / 4)) * 4;
            const int gr = m0 + r, gk = k0 + kq;
            ra[v] = (gr < g.M && gk < g.lda) ? *(const float4*)(A + (int64_t)gr * g.lda + gk)
                                             : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int v = 0; v < VB; ++v) {
            const int idx = tid + v * 256;
            const int r = idx / (BK / 4), kq = (idx % (BK / 4)) * 4;
            const int gr = n0 + r, gk = k0 + kq;
            rb[v] = (gr < g.N && gk < g.ldb) ? *(const float4*)(B + (int64_t)gr * g.ldb + gk)
                                             : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int v = 0; v < VA; ++v) {
            const int idx = tid + v * 256;
            const int r = idx / (BK / 4), kq = (idx % (BK / 4)) * 4;
            float* d = &As[r * LDF + kq];
            d[0] = ra[v].x;
            d[1] = ra[v].y;
            d[2] = ra[v].z;
            d[3] = ra[v].w;
        }
#pragma unroll
        for (int v = 0; v < VB; ++v) {
            const int idx = tid + v * 256;
            const int r = idx / (BK / 4), kq = (idx % (BK / 4)) * 4;
            float* d = &Bs[r * LDF + kq];
            d[0] = rb[v].x;
            d[1] = rb[v].y;
            d[2] = rb[v].z;
            d[3] = rb[v].w;
        }
    };

    f16_t acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

    const int kb = tw.k0, ke = tw.k1;   // this item's K range (whole stages but the last)
    if (ke > kb) gload(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        sstore();
        __syncthreads();
        if (k0 + BK < ke) gload(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 2) {
            float a[TI], b[TJ];
#pragma unroll
            for (int i = 0; i < TI; ++i) a[i] = As[(wm + i * 32 + (lane & 31)) * LDF + kk + (lane >> 5)];
#pragma unroll
            for (int j = 0; j < TJ; ++j) b[j] = Bs[(wn + j * 32 + (lane & 31)) * LDF + kk + (lane >> 5)];
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // a whole-K item writes C; a split-K part writes its partial tile
    float* __restrict__ W = ws + (int64_t)(tw.slot < 0 ? 0 : tw.slot) * BM * BN;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int col = n0 + wn + j * 32 + (lane & 31);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = m0 + wm + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                if (tw.slot >= 0) W[(row - m0) * BN + (col - n0)] = acc[i][j][e];
                else if (row < g.M && col < g.N) C[(int64_t)row * g.ldc + col] = acc[i][j][e];
            }
        }
    }
    if (!queue) break;
    if (threadIdx.x == 0) next_row = (int)(gridDim.x >> 3) + atomicAdd(&queue[blockIdx.x & 7], 1);
    __syncthreads();
    t = next_row * 8 + (int)(blockIdx.x & 7);
    __syncthreads();
  }
}

// ---- BF16 panels: v_mfma_f32_32x32x16_bf16 ---------------------------------
// The gather has already rounded (BF16, PL = 1) or split (BF16X3, PL = 2:
// hi and lo planes; BF16X6, PL = 3: hi, mid and lo planes, plane p at
// p * a_lo / p * b_lo elements) the operands, so tiles go global -> LDS as
// 16-byte vectors with no conversion.  The split products are accumulated in
// FP32, smallest terms first: bf16x3 = lo*hi + hi*lo + hi*hi; bf16x6 =
// lo*hi + hi*lo + mid*mid + mid*hi + hi*mid + hi*hi (the dropped mid*lo,
// lo*mid, lo*lo are below FP32 rounding of the product).
template <class Ptrs, class S, int PL, bool SCAT>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const TileWork* __restrict__ tiles, int ntiles,
                                                        int* __restrict__ queue,
                                                        const GemmGroup* __restrict__ groups, Ptrs ptrs,
                                                        float* __restrict__ ws) {
    constexpr int BM = S::BM, BN = S::BN, BK = S::BK;
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TI = WM / 32, TJ = WN / 32;
    constexpr int LDH = BK + 8;
    static_assert(PL >= 1 && PL <= 3, "one to three bf16 planes");
    static_assert(TI >= 1 && TJ >= 1 && BK % 16 == 0, "tile shape");
    // one LDS region: the A and B tiles of the K loop; the scatter
    // epilogue's tables and staged products afterwards
    __shared__ __attribute__((aligned(16))) unsigned short smem[PL * (BM + BN) * LDH];
    unsigned short (*As)[BM * LDH] = reinterpret_cast<unsigned short (*)[BM * LDH]>(smem);
    unsigned short (*Bs)[BN * LDH] = reinterpret_cast<unsigned short (*)[BN * LDH]>(smem + PL * BM * LDH);

  // Entry t of the list belongs to XCD t mod 8, and workgroup b runs on XCD
  // b mod 8.  Each workgroup starts with its own entry; with a queue (a
  // persistent grid smaller than the list), it then takes the next free row
  // of its XCD's list from that XCD's counter.
  __shared__ int next_row;
  for (int t = blockIdx.x; t < ntiles;) {
    const TileWork tw = tiles[t];
    if (tw.group >= 0) {   // group < 0: padding of the per-XCD lists
    const GemmGroup g = groups[tw.group];
    const unsigned short* __restrict__ A = (const unsigned short*)ptrs.get(g.a_buf) + g.a_off;
    const unsigned short* __restrict__ B = (const unsigned short*)ptrs.get(g.b_buf) + g.b_off;
    float* __restrict__ C = (float*)ptrs.get(g.c_buf) + g.c_off;
    const int m0 = tw.tm * BM, n0 = tw.tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

    constexpr int VA = BM * BK / 8 / 256;   // 16-byte vectors per thread and plane
    constexpr int VB = BN * BK / 8 / 256;
    static_assert(VA >= 1 && VB >= 1, "tile too small");
    us8_t ra[PL][VA], rb[PL][VB];
    const us8_t zero8 = {0, 0, 0, 0, 0, 0, 0, 0};

    auto gload = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PL; ++p) {
#pragma unroll
            for (int v = 0; v < VA; ++v) {
                const int idx = tid + v * 256;
                const int r = idx / (BK / 8), kq = (idx % (BK / 8)) * 8;
                const int gr = m0 + r, gk = k0 + kq;
                ra[p][v] = (gr < g.M && gk < g.lda)
                               ? *(const us8_t*)(A + p * g.a_lo + (int64_t)gr * g.lda + gk)
                               : zero8;
            }
#pragma unroll
            for (int v = 0; v < VB; ++v) {
                const int idx = tid + v * 256;
                const int r = idx / (BK / 8), kq = (idx % (BK / 8)) * 8;
                const int gr = n0 + r, gk = k0 + kq;
                rb[p][v] = (gr < g.N && gk < g.ldb)
                               ? *(const us8_t*)(B + p * g.b_lo + (int64_t)gr * g.ldb + gk)
                               : zero8;
            }
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int p = 0; p < PL; ++p) {
#pragma unroll
            for (int v = 0; v < VA; ++v) {
                const int idx = tid + v * 256;
                const int r = idx / (BK / 8), kq = (idx % (BK / 8)) * 8;
                *(us8_t*)(&As[p][r * LDH + kq]) = ra[p][v];
            }
#pragma unroll
            for (int v = 0; v < VB; ++v) {
                const int idx = tid + v * 256;
                const int r = idx / (BK / 8), kq = (idx % (BK / 8)) * 8;
                *(us8_t*)(&Bs[p][r * LDH + kq]) = rb[p][v];
            }
        }
    };

    f16_t acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

    const int kb = tw.k0, ke = tw.k1;   // this item's K range (whole stages but the last)
    if (ke > kb) gload(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        sstore();
        __syncthreads();
        if (k0 + BK < ke) gload(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            // plane 0 = hi, PL - 1 = lo, 1 = mid (PL = 3)
            bf8_t ah[TI], bh[TJ], al[TI], bl[TJ], am[TI], bm[TJ];
#pragma unroll
            for (int i = 0; i < TI; ++i) {
                const int o = (wm + i * 32 + (lane & 31)) * LDH + kk + 8 * (lane >> 5);
                ah[i] = __builtin_bit_cast(bf8_t, *(const us8_t*)(&As[0][o]));
                if constexpr (PL > 1) al[i] = __builtin_bit_cast(bf8_t, *(const us8_t*)(&As[PL - 1][o]));
                if constexpr (PL > 2) am[i] = __builtin_bit_cast(bf8_t, *(const us8_t*)(&As[1][o]));
            }
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const int o = (wn + j * 32 + (lane & 31)) * LDH + kk + 8 * (lane >> 5);
                bh[j] = __builtin_bit_cast(bf8_t, *(const us8_t*)(&Bs[0][o]));
                if constexpr (PL > 1) bl[j] = __builtin_bit_cast(bf8_t, *(const us8_t*)(&Bs[PL - 1][o]));
                if constexpr (PL > 2) bm[j] = __builtin_bit_cast(bf8_t, *(const us8_t*)(&Bs[1][o]));
            }
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j) {
                    if constexpr (PL > 1) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    }
                    if constexpr (PL > 2) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am[i], bm[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am[i], bh[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bm[j], acc[i][j], 0, 0, 0);
                    }
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    if constexpr (SCAT) {
        // scatter epilogue (never split along K): each product goes, split
        // into this kernel's bf16 planes, to the position the next
        // contraction's A panel holds it at.  The tile's row and column
        // entries and the block entries they meet are staged in LDS (the A
        // tile's space, free after the K loop), so that the epilogue's
        // global memory operations are its stores.  A lane holds four
        // consecutive rows of a column; where they land on four
        // consecutive, aligned positions they are stored as one vector per
        // plane.
        const int* __restrict__ tab = (const int*)ptrs.get(g.s_buf);
        const int* __restrict__ rt = tab + g.s_rows;
        const int* __restrict__ ct = tab + g.s_cols;
        const int* __restrict__ bt = tab + g.s_blocks;
        unsigned short* __restrict__ P = (unsigned short*)ptrs.get(g.c_buf);
        constexpr int kLdsInts = PL * BM * LDH / 2;
        constexpr int kMaxBlk = (kLdsInts - 4 * (BM + BN)) / 8;
        static_assert(kMaxBlk >= 16, "LDS too small for the scatter tables");
        int* srow = (int*)&As[0][0];
        int* scol = srow + 4 * BM;
        int* sblk = scol + 4 * BN;
        const int mlast = min(m0 + BM, g.M) - 1, nlast = min(n0 + BN, g.N) - 1;
        const int rb_lo = rt[4 * m0], rb_hi = rt[4 * mlast];   // rows are ordered by row block
        const int cb_lo = ct[4 * n0], cb_hi = ct[4 * nlast];
        const int ncbt = cb_hi - cb_lo + 1;
        const bool staged = (rb_hi - rb_lo + 1) * ncbt <= kMaxBlk;
        __syncthreads();   // every wave is done with the A and B tiles
        for (int e = tid; e < BM; e += 256)
            if (m0 + e <= mlast) *(int4*)(srow + 4 * e) = *(const int4*)(rt + 4 * (m0 + e));
        for (int e = tid; e < BN; e += 256)
            if (n0 + e <= nlast) *(int4*)(scol + 4 * e) = *(const int4*)(ct + 4 * (n0 + e));
        if (staged)
            for (int e = tid; e < (rb_hi - rb_lo + 1) * ncbt; e += 256) {
                const int* src = bt + 8 * ((rb_lo + e / ncbt) * g.s_ncb + cb_lo + e % ncbt);
                *(int4*)(sblk + 8 * e) = *(const int4*)src;
                *(int4*)(sblk + 8 * e + 4) = *(const int4*)(src + 4);
            }
        __syncthreads();
        auto entry = [&](int rb, int cb, int4& b0, int4& b1) {
            if (staged) {
                const int* e = sblk + 8 * ((rb - rb_lo) * ncbt + (cb - cb_lo));
                b0 = *(const int4*)e;
                b1 = *(const int4*)(e + 4);
            } else {
                const int* e = bt + 8 * (rb * g.s_ncb + cb);
                b0 = *(const int4*)e;
                b1 = *(const int4*)(e + 4);
            }
        };
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int cl = wn + j * 32 + (lane & 31);
            if (n0 + cl >= g.N) continue;
            const int4 cr = *(const int4*)(scol + 4 * cl);
#pragma unroll
            for (int i = 0; i < TI; ++i) {
                // the block entry of the sub-tile's first row; rows of another
                // row block look theirs up
                const int rl0 = wm + i * 32;
                const int rb0 = srow[4 * min(rl0, mlast - m0)];
                int4 c0, c1;
                entry(rb0, cr.x, c0, c1);
#pragma unroll
                for (int eg = 0; eg < 4; ++eg) {
                    const int rl = rl0 + 8 * eg + 4 * (lane >> 5);
                    int d[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        d[q] = -1;
                        if (m0 + rl + q > mlast) continue;
                        const int4 rr = *(const int4*)(srow + 4 * (rl + q));
                        int4 b0 = c0, b1 = c1;
                        if (rr.x != rb0) entry(rr.x, cr.x, b0, b1);
                        if (b0.x >= 0)
                            d[q] = b0.x + rr.y * b0.y + rr.z * b0.z + rr.w * b0.w + cr.y * b1.x + cr.z * b1.y +
                                   cr.w * b1.z;
                    }
                    unsigned short h[4][3];
#pragma unroll
                    for (int q = 0; q < 4; ++q) bf16_planes<PL>(acc[i][j][4 * eg + q], h[q]);
                    if (d[0] >= 0 && (d[0] & 3) == 0 && d[1] == d[0] + 1 && d[2] == d[0] + 2 && d[3] == d[0] + 3) {
#pragma unroll
                        for (int p = 0; p < PL; ++p) {
                            const uint2 v = {(uint32_t)h[0][p] | ((uint32_t)h[1][p] << 16),
                                             (uint32_t)h[2][p] | ((uint32_t)h[3][p] << 16)};
                            *(uint2*)(P + d[0] + p * g.c_lo) = v;
                        }
                    } else {
                        // pairs of consecutive, aligned positions as one 4-byte store
#pragma unroll
                        for (int q = 0; q < 4; q += 2) {
                            if (d[q] >= 0 && (d[q] & 1) == 0 && d[q + 1] == d[q] + 1) {
#pragma unroll
                                for (int p = 0; p < PL; ++p)
                                    *(uint32_t*)(P + d[q] + p * g.c_lo) =
                                        (uint32_t)h[q][p] | ((uint32_t)h[q + 1][p] << 16);
                            } else {
#pragma unroll
                                for (int k = q; k < q + 2; ++k)
                                    if (d[k] >= 0)
#pragma unroll
                                        for (int p = 0; p < PL; ++p) P[d[k] + p * g.c_lo] = h[k][p];
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();   // the LDS tables are read before the next tile's loads
    } else {
    // a whole-K item writes C; a split-K part writes its partial tile
    float* __restrict__ W = ws + (int64_t)(tw.slot < 0 ? 0 : tw.slot) * BM * BN;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int col = n0 + wn + j * 32 + (lane & 31);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = m0 + wm + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                if (tw.slot >= 0) W[(row - m0) * BN + (col - n0)] = acc[i][j][e];
                else if (row < g.M && col < g.N) C[(int64_t)row * g.ldc + col] = acc[i][j][e];
            }
        }
    }
    }
    if (!queue) break;
    if (threadIdx.x == 0) next_row = (int)(gridDim.x >> 3) + atomicAdd(&queue[blockIdx.x & 7], 1);
    __syncthreads();
    t = next_row * 8 + (int)(blockIdx.x & 7);
    __syncthreads();
  }
}

// Split K: every output tile of `outs` is the sum of its parts' partial
// tiles (workspace slots slot0 .. slot0 + nparts - 1), added in part order.
template <class Ptrs, typename T>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const SplitOut* __restrict__ outs,
                                                            const GemmGroup* __restrict__ groups, Ptrs ptrs,
                                                            const T* __restrict__ ws, int BM, int BN) {
    const SplitOut so = outs[blockIdx.x];
    const GemmGroup g = groups[so.group];
    T* __restrict__ C = (T*)ptrs.get(g.c_buf) + g.c_off;
    const int64_t tile = (int64_t)BM * BN;
    for (int e = threadIdx.x; e < BM * BN; e += 256) {
        const int row = so.tm * BM + e / BN, col = so.tn * BN + e % BN;
        if (row >= g.M || col >= g.N) continue;
        T sum = ws[so.slot0 * tile + e];
        for (int p = 1; p < so.nparts; ++p) sum += ws[(so.slot0 + p) * tile + e];
        C[(int64_t)row * g.ldc + col] = sum;
    }
}

// ================================================================ utilities
__global__ void cast_kernel_d2f(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (float)s[i];
}
__global__ void cast_kernel_f2d(const float* __restrict__ s, double* __restrict__ d, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (double)s[i];
}
// One entry of a device pointer table, written in stream order (a replayed
// HIP graph reads its buffers through such a table).
__global__ void set_pointer_kernel(void** __restrict__ table, int idx, void* p) {
    if (threadIdx.x == 0) table[idx] = p;
}
__global__ void fill_zero_kernel(uint32_t* __restrict__ d, int64_t nwords) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = 0u;
}

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 512;

template <typename T>
__global__ __launch_bounds__(kRedThreads) void sumsq_partial_kernel(const T* __restrict__ x, int64_t n,
                                                                    double* __restrict__ partial) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads) {
        const double v = (double)x[i];
        s = fma(v, v, s);
    }
    // wavefront reduction (64 lanes) then across the 4 waves via LDS
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    __shared__ double ws[kRedThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w) t += ws[w];
        partial[blockIdx.x] = t;
    }
}
__global__ __launch_bounds__(kRedThreads) void sum_final_kernel(const double* __restrict__ partial, int n,
                                                                double* __restrict__ out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kRedThreads) s += partial[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    __shared__ double ws[kRedThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w) t += ws[w];
        *out = t;
    }
}
template <typename T>
__global__ void scale_inv_sqrt_kernel(T* __restrict__ x, int64_t n, const double* __restrict__ sumsq) {
    const double s = *sumsq;
    const double f = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = (T)((double)x[i] * f);
}

// Projector sign gauge: for each row j of P~ (col-major, ld ldPt, n cols)
// find the largest |entry| (lowest column on ties); if it is negative, flip
// row j of P~ and column j of P (col-major, ld ldP).
__global__ __launch_bounds__(256) void sign_fix_kernel(double* __restrict__ Pt, int ldPt, int n,
                                                       double* __restrict__ P, int ldP) {
    const int j = blockIdx.x;
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int f = threadIdx.x; f < n; f += 256) {
        const double v = fabs(Pt[j + (int64_t)f * ldPt]);
        if (v > best || (v == best && f < bi)) { best = v; bi = f; }
    }
    __shared__ double sb[256];
    __shared__ int si[256];
    sb[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double ob = sb[threadIdx.x + s];
            const int oi = si[threadIdx.x + s];
            if (ob > sb[threadIdx.x] || (ob == sb[threadIdx.x] && oi < si[threadIdx.x])) {
                sb[threadIdx.x] = ob;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int arg = si[0];
    const bool flip = arg < n && Pt[j + (int64_t)arg * ldPt] < 0.0;
    __syncthreads();
    if (flip) {
        for (int f = threadIdx.x; f < n; f += 256) {
            Pt[j + (int64_t)f * ldPt] = -Pt[j + (int64_t)f * ldPt];
            P[(int64_t)j * ldP + f] = -P[(int64_t)j * ldP + f];
        }
    }
}

// Double layer: thread per output element.  Output blocks are contiguous
// row-major in canonical order; per leg a fused state maps to (ket, bra)
// states of the virtual leg.
template <typename T>
__global__ __launch_bounds__(256) void double_layer_kernel(DoubleLayerArgs a) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.total) return;
    int lo = 0, hi = a.nblocks - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.blk_elem_start[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const int b = lo;
    int64_t r = i - a.blk_elem_start[b];
    int f[4];
#pragma unroll
    for (int l = 3; l >= 0; --l) {
        const int d = a.blk_shape[b * 4 + l];
        f[l] = a.blk_start[b * 4 + l] + (int)(r % d);
        r /= d;
    }
    int k[4], br[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        k[l] = a.ket_of[l][f[l]];
        br[l] = a.bra_of[l][f[l]];
    }
    const T* __restrict__ Ad = (const T*)a.A_dense;
    const int64_t s1 = a.Dv[3], s2 = s1 * a.Dv[2], s3 = s2 * a.Dv[1], s4 = s3 * a.Dv[0];
    const int64_t ok = k[0] * s3 + k[1] * s2 + k[2] * s1 + k[3];
    const int64_t ob = br[0] * s3 + br[1] * s2 + br[2] * s1 + br[3];
    double acc = 0.0;
    if (!a.has_op) {
        for (int s = 0; s < a.nphys; ++s) acc = fma((double)Ad[s * s4 + ok], (double)Ad[s * s4 + ob], acc);
    } else {
        for (int sb = 0; sb < a.nphys; ++sb) {
            double row = 0.0;
            for (int sk = 0; sk < a.nphys; ++sk) row = fma(a.op[sb * a.nphys + sk], (double)Ad[sk * s4 + ok], row);
            acc = fma(row, (double)Ad[sb * s4 + ob], acc);
        }
    }
    ((T*)a.out)[a.blk_off[b] + (i - a.blk_elem_start[b])] = (T)acc;
}

// ============================================================ host launchers
namespace {
inline int grid_for(int64_t n, int threads, int cap = 65535 * 4) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}
}  // namespace

void launch_cast(const void* src, bool src_f64, void* dst, bool dst_f64, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int g = grid_for(n, 256, 8192);
    if (src_f64 && !dst_f64)
        hipLaunchKernelGGL(cast_kernel_d2f, dim3(g), dim3(256), 0, s, (const double*)src, (float*)dst, n);
    else if (!src_f64 && dst_f64)
        hipLaunchKernelGGL(cast_kernel_f2d, dim3(g), dim3(256), 0, s, (const float*)src, (double*)dst, n);
    else
        HIPCHK(hipMemcpyAsync(dst, src, n * (src_f64 ? 8 : 4), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipGetLastError());
}

void launch_set_pointer(void** table, int idx, void* p, hipStream_t s) {
    hipLaunchKernelGGL(set_pointer_kernel, dim3(1), dim3(64), 0, s, table, idx, p);
    HIPCHK(hipGetLastError());
}

void launch_fill_zero(void* dst, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return;
    if (bytes % 4) fail(SYMTEN_E_INVAL, "fill_zero: size not a multiple of 4 bytes");
    const int64_t nw = bytes / 4;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(nw, 256, 8192)), dim3(256), 0, s, (uint32_t*)dst, nw);
    HIPCHK(hipGetLastError());
}

void launch_sumsq(const void* x, bool f64, int64_t n, double* out, hipStream_t s) {
    // partial sums live right after *out (caller provides 1 + kRedBlocks doubles)
    double* partial = out + 1;
    const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + kRedThreads - 1) / kRedThreads));
    if (f64)
        hipLaunchKernelGGL(sumsq_partial_kernel<double>, dim3(nb), dim3(kRedThreads), 0, s, (const double*)x, n, partial);
    else
        hipLaunchKernelGGL(sumsq_partial_kernel<float>, dim3(nb), dim3(kRedThreads), 0, s, (const float*)x, n, partial);
    hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(kRedThreads), 0, s, (const double*)partial, nb, out);
    HIPCHK(hipGetLastError());
}

void launch_scale_by_inv_sqrt(void* x, bool f64, int64_t n, const double* sumsq, hipStream_t s) {
    if (n <= 0) return;
    const int g = grid_for(n, 256, 8192);
    if (f64)
        hipLaunchKernelGGL(scale_inv_sqrt_kernel<double>, dim3(g), dim3(256), 0, s, (double*)x, n, sumsq);
    else
        hipLaunchKernelGGL(scale_inv_sqrt_kernel<float>, dim3(g), dim3(256), 0, s, (float*)x, n, sumsq);
    HIPCHK(hipGetLastError());
}

void launch_sign_fix_rows(double* Pt, int ldPt, int rows, int n, double* P, int ldP, hipStream_t s) {
    if (rows <= 0 || n <= 0) return;
    hipLaunchKernelGGL(sign_fix_kernel, dim3(rows), dim3(256), 0, s, Pt, ldPt, n, P, ldP);
    HIPCHK(hipGetLastError());
}

void launch_double_layer(const DoubleLayerArgs& a, hipStream_t s) {
    if (a.total <= 0) return;
    const int64_t g = (a.total + 255) / 256;
    if (a.f64)
        hipLaunchKernelGGL(double_layer_kernel<double>, dim3((unsigned)g), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(double_layer_kernel<float>, dim3((unsigned)g), dim3(256), 0, s, a);
    HIPCHK(hipGetLastError());
}

// ---- prepared launches: device descriptors owned by the caller ------------
template <class Ptrs>
static void copy_dispatch(const CopyTask* d_tasks, const int64_t* d_prefix, int ntasks, int64_t npieces, Ptrs P,
                          bool src_f64, int dst_kind, hipStream_t s) {
    dim3 grid((unsigned)npieces), block(kCopyThreads);
#define SYMTEN_COPY(TS, DK) \
    hipLaunchKernelGGL((copy_kernel<Ptrs, TS, DK>), grid, block, 0, s, d_tasks, d_prefix, ntasks, P)
    if (src_f64) {
        switch (dst_kind) {
            case kDstF64: SYMTEN_COPY(double, kDstF64); break;
            case kDstF32: SYMTEN_COPY(double, kDstF32); break;
            case kDstAcc: SYMTEN_COPY(double, kDstAcc); break;
            default: fail(SYMTEN_E_INVAL, "copy: bf16 panels need FP32 sources");
        }
    } else {
        switch (dst_kind) {
            case kDstF64: SYMTEN_COPY(float, kDstF64); break;
            case kDstF32: SYMTEN_COPY(float, kDstF32); break;
            case kDstBF16: SYMTEN_COPY(float, kDstBF16); break;
            case kDstAcc: SYMTEN_COPY(float, kDstAcc); break;
            case kDstSplit: SYMTEN_COPY(float, kDstSplit); break;
            case kDstSplit3: SYMTEN_COPY(float, kDstSplit3); break;
            default: fail(SYMTEN_E_INVAL, "copy: unknown destination kind");
        }
    }
#undef SYMTEN_COPY
    HIPCHK(hipGetLastError());
}

void copy_launch_dev(const CopyTask* d_tasks, const int64_t* d_prefix, int ntasks, int64_t npieces,
                     void* const* d_ptrs, bool src_f64, int dst_kind, hipStream_t s) {
    if (ntasks <= 0 || npieces <= 0) return;
    copy_dispatch(d_tasks, d_prefix, ntasks, npieces, DevPtrs{d_ptrs}, src_f64, dst_kind, s);
}

void copy_launch_arg(const CopyTask* d_tasks, const int64_t* d_prefix, int ntasks, int64_t npieces,
                     const std::vector<void*>& ptrs, bool src_f64, int dst_kind, hipStream_t s) {
    if (ntasks <= 0 || npieces <= 0) return;
    if (ptrs.size() > 16) fail(SYMTEN_E_CAPACITY, "copy_launch_arg: more than 16 buffers");
    ArgPtrs P{};
    for (size_t i = 0; i < ptrs.size(); ++i) P.p[i] = ptrs[i];
    copy_dispatch(d_tasks, d_prefix, ntasks, npieces, P, src_f64, dst_kind, s);
}

// Tile shapes (BM x BN): 0 = 64x64, 1 = 128x128, 2 = 128x64, 3 = 64x128,
// 4 = 256x128 (FP32/BF16 kernels only), and with twice the K depth per
// stage (more MFMA work between a stage's loads and their use, for launches
// of few tiles per CU): 5 = 64x64, 6 = 128x64, 7 = 64x128.  K depth: FP64
// 16 (32 for 5-7), FP32/BF16 32 (64 for 5-7).
static const int kTileBM[kNumTileCfg] = {64, 128, 128, 64, 256, 64, 128, 64};
static const int kTileBN[kNumTileCfg] = {64, 128, 64, 128, 128, 64, 64, 128};
int gemm_tile_bm(Prec p, int cfg) { (void)p; return kTileBM[cfg]; }
int gemm_tile_bn(Prec p, int cfg) { (void)p; return kTileBN[cfg]; }
int gemm_tile_bk(Prec p, int cfg) { return (p == Prec::F64 ? 16 : 32) * (cfg >= 5 ? 2 : 1); }
bool gemm_tile_ok(Prec p, int cfg) { return cfg >= 0 && cfg < kNumTileCfg && !(p == Prec::F64 && cfg == 4); }

// Kernel of a (precision, tile configuration); FP32, BF16, bf16x3 and
// bf16x6 accumulate in FP32, FP64 in FP64.
template <class Ptrs>
using GemmF64Fn = void (*)(const TileWork*, int, int*, const GemmGroup*, Ptrs, double*);
template <class Ptrs>
using GemmF32Fn = void (*)(const TileWork*, int, int*, const GemmGroup*, Ptrs, float*);

template <class Ptrs>
static GemmF64Fn<Ptrs> f64_kernel(int cfg) {
    switch (cfg) {
        case 0: return gemm_f64_kernel<Ptrs, TileShape<64, 64, 16>>;
        case 1: return gemm_f64_kernel<Ptrs, TileShape<128, 128, 16>>;
        case 2: return gemm_f64_kernel<Ptrs, TileShape<128, 64, 16>>;
        case 3: return gemm_f64_kernel<Ptrs, TileShape<64, 128, 16>>;
        case 5: return gemm_f64_kernel<Ptrs, TileShape<64, 64, 32>>;
        case 6: return gemm_f64_kernel<Ptrs, TileShape<128, 64, 32>>;
        default: return gemm_f64_kernel<Ptrs, TileShape<64, 128, 32>>;
    }
}

template <class Ptrs, int PL, bool SCAT>
static GemmF32Fn<Ptrs> bf16_kernel(int cfg) {
    switch (cfg) {
        case 0: return gemm_bf16_kernel<Ptrs, TileShape<64, 64, 32>, PL, SCAT>;
        case 1: return gemm_bf16_kernel<Ptrs, TileShape<128, 128, 32>, PL, SCAT>;
        case 2: return gemm_bf16_kernel<Ptrs, TileShape<128, 64, 32>, PL, SCAT>;
        case 3: return gemm_bf16_kernel<Ptrs, TileShape<64, 128, 32>, PL, SCAT>;
        case 4: return gemm_bf16_kernel<Ptrs, TileShape<256, 128, 32>, PL, SCAT>;
        case 5: return gemm_bf16_kernel<Ptrs, TileShape<64, 64, 64>, PL, SCAT>;
        case 6: return gemm_bf16_kernel<Ptrs, TileShape<128, 64, 64>, PL, SCAT>;
        default: return gemm_bf16_kernel<Ptrs, TileShape<64, 128, 64>, PL, SCAT>;
    }
}

// scatter: the kernel with the scatter epilogue (bf16 precisions only)
template <class Ptrs>
static GemmF32Fn<Ptrs> f32_kernel(Prec p, int cfg, bool scatter = false) {
    switch (p) {
        case Prec::BF16: return scatter ? bf16_kernel<Ptrs, 1, true>(cfg) : bf16_kernel<Ptrs, 1, false>(cfg);
        case Prec::BF16X3: return scatter ? bf16_kernel<Ptrs, 2, true>(cfg) : bf16_kernel<Ptrs, 2, false>(cfg);
        case Prec::BF16X6: return scatter ? bf16_kernel<Ptrs, 3, true>(cfg) : bf16_kernel<Ptrs, 3, false>(cfg);
        default: break;
    }
    if (scatter) fail(SYMTEN_E_INVAL, "gemm: the scatter epilogue needs a bf16 precision");
    switch (cfg) {
        case 0: return gemm_f32_kernel<Ptrs, TileShape<64, 64, 32>>;
        case 1: return gemm_f32_kernel<Ptrs, TileShape<128, 128, 32>>;
        case 2: return gemm_f32_kernel<Ptrs, TileShape<128, 64, 32>>;
        case 3: return gemm_f32_kernel<Ptrs, TileShape<64, 128, 32>>;
        case 4: return gemm_f32_kernel<Ptrs, TileShape<256, 128, 32>>;
        case 5: return gemm_f32_kernel<Ptrs, TileShape<64, 64, 64>>;
        case 6: return gemm_f32_kernel<Ptrs, TileShape<128, 64, 64>>;
        default: return gemm_f32_kernel<Ptrs, TileShape<64, 128, 64>>;
    }
}

bool gemm_persistent(int ntiles, int capacity) { return ntiles > kPersistentFactor * capacity; }

// Workgroups of a (precision, tile) kernel that the chip runs at once: its
// occupancy per compute unit times the compute units (a multiple of the 8
// XCDs), measured once per device and kernel.
int gemm_capacity(Prec p, int cfg) {
    if (!gemm_tile_ok(p, cfg)) fail(SYMTEN_E_INVAL, "gemm: tile configuration not available");
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static int cache[kMaxDev][5][kNumTileCfg] = {};
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) fail(SYMTEN_E_CAPACITY, "gemm: device index beyond 63");
    std::lock_guard<std::mutex> lk(mu);
    int& c = cache[dev][(int)p][cfg];
    if (c == 0) {
        int cus = 0, per_cu = 0;
        HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const void* fn = p == Prec::F64 ? (const void*)f64_kernel<DevPtrs>(cfg) : (const void*)f32_kernel<DevPtrs>(p, cfg);
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0));
        c = std::max(8, std::max(1, per_cu) * std::max(1, cus) / 8 * 8);
    }
    return c;
}

template <class Ptrs>
static void gemm_dispatch(const TileWork* d_tiles, int ntiles, const GemmGroup* d_groups, Ptrs P, Prec prec,
                          int cfg, hipStream_t s, const SplitK& sk, bool scatter) {
    if (!gemm_tile_ok(prec, cfg)) fail(SYMTEN_E_INVAL, "gemm: tile configuration not available");
    if (scatter && sk.nsplits > 0) fail(SYMTEN_E_INVAL, "gemm: the scatter epilogue is not split along K");
    // persistent grid for long lists: as many workgroups as the chip holds at
    // once, taking further entries from per-XCD counters (the first
    // kSplitQueueBytes of the workspace, zeroed here in stream order); a list
    // up to kPersistentFactor times the capacity is left to the
    // hardware dispatcher (measured as fast, one launch less)
    const int cap = gemm_capacity(prec, cfg);
    const bool persistent = gemm_persistent(ntiles, cap);
    if ((sk.nsplits > 0 || persistent) && !sk.ws) fail(SYMTEN_E_INVAL, "gemm: no workspace for the queue or split K");
    if (sk.nsplits > 0 && !sk.splits) fail(SYMTEN_E_INVAL, "gemm: split K without its output list");
    int* queue = persistent ? (int*)sk.ws : nullptr;
    void* partials = sk.ws ? (char*)sk.ws + kSplitQueueBytes : nullptr;
    if (persistent) launch_fill_zero(queue, 8 * sizeof(int), s);
    const dim3 grid((unsigned)(persistent ? cap : ntiles)), block(256);
    if (prec == Prec::F64)
        hipLaunchKernelGGL(f64_kernel<Ptrs>(cfg), grid, block, 0, s, d_tiles, ntiles, queue, d_groups, P,
                           (double*)partials);
    else
        hipLaunchKernelGGL(f32_kernel<Ptrs>(prec, cfg, scatter), grid, block, 0, s, d_tiles, ntiles, queue, d_groups,
                           P, (float*)partials);
    HIPCHK(hipGetLastError());
    if (sk.nsplits > 0) {
        const int BM = gemm_tile_bm(prec, cfg), BN = gemm_tile_bn(prec, cfg);
        if (prec == Prec::F64)
            hipLaunchKernelGGL((splitk_reduce_kernel<Ptrs, double>), dim3(sk.nsplits), dim3(256), 0, s, sk.splits,
                               d_groups, P, (const double*)partials, BM, BN);
        else
            hipLaunchKernelGGL((splitk_reduce_kernel<Ptrs, float>), dim3(sk.nsplits), dim3(256), 0, s, sk.splits,
                               d_groups, P, (const float*)partials, BM, BN);
        HIPCHK(hipGetLastError());
    }
}

void gemm_launch_arg(const TileWork* d_tiles, int ntiles, const GemmGroup* d_groups,
                     const std::vector<void*>& ptrs, Prec prec, int cfg, hipStream_t s, const SplitK& sk) {
    if (ntiles <= 0) return;
    if (ptrs.size() > 16) fail(SYMTEN_E_CAPACITY, "gemm_launch_arg: more than 16 buffers");
    ArgPtrs P{};
    for (size_t i = 0; i < ptrs.size(); ++i) P.p[i] = ptrs[i];
    gemm_dispatch(d_tiles, ntiles, d_groups, P, prec, cfg, s, sk, false);
}

void gemm_launch_dev(const TileWork* d_tiles, int ntiles, const GemmGroup* d_groups, void* const* d_ptrs,
                     Prec prec, int cfg, hipStream_t s, const SplitK& sk, bool scatter) {
    if (ntiles <= 0) return;
    gemm_dispatch(d_tiles, ntiles, d_groups, DevPtrs{d_ptrs}, prec, cfg, s, sk, scatter);
}

}  // namespace symten
