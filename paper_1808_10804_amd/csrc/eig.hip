// FP64 symmetric eigensolver of the projector stage (Sec. 3: the projectors
// of the scheme it cites come from the singular triplets of one matrix per
// sector of the cut; here they are taken from a symmetric eigenproblem, the
// Gram matrix Y Y^T or the Jordan-Wielandt matrix [[0, Y], [Y^T, 0]]).
//
// Four steps, each one launch over every matrix of a cut:
//   1. Householder tridiagonalisation T = Q^T A Q (Q = H_0 ... H_{n-3},
//      H_k = I - tau_k v_k v_k^T).  The rows of a matrix are spread over the
//      workgroups of one job, cyclically (row i on workgroup i mod G), and
//      stay in LDS for the whole reduction.  The rank-2 update of column k,
//      A -= v w^T + w v^T, is applied lazily: each workgroup applies it to
//      its own rows in the pass of column k+1 that also forms p = tau A v, so
//      one column costs one exchange between the job's workgroups (its p
//      slices and the next row, through global memory, then a barrier on an
//      atomic counter).  The jobs of a launch sit on disjoint workgroups,
//      each job on the workgroups of one XCD where it fits.
//   2. All eigenvalues by multisection: one wavefront per eigenvalue, its 64
//      lanes evaluating Sturm counts of T at 64 points of the current
//      interval, about 9 passes to 2 ulp.
//   3. Eigenvectors of T for the kept eigenvalues from the twisted
//      factorisation of T - lam I (two recurrences, no iteration; for an
//      eigenvalue apart from the others both run at once).  Eigenvalues
//      closer than 1e-3 ||T|| form a cluster, done in order by one
//      wavefront: each vector has the earlier ones projected out, and if
//      less than half of it is left (a degenerate value) it comes from
//      inverse iteration instead (tridiagonal LU with partial pivoting, two
//      solves from a fixed pseudo-random start, reorthogonalised in every
//      solve).
//   4. Back-transformation z <- Q z through the stored reflectors, one
//      vector per workgroup held in LDS, one block-wide reduction per
//      reflector, the reflectors streamed through LDS in chunks.
// The matrix is scaled by a power of two (exact) so that its largest entry
// is in [1, 2); eigenvalues are returned unscaled.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "internal.hpp"

namespace symten {
namespace {

constexpr int kEigThreads = 256;                 // bisection: four eigenvalues per workgroup
constexpr int kEigWaves = kEigThreads / 64;
// Tridiagonalisation and back-transformation: one workgroup per compute unit
// (their LDS), so 1024 threads give each SIMD four waves to hide LDS and
// FP64 latency with.
constexpr int kTriThreads = 1024;
constexpr int kTriWaves = kTriThreads / 64;
constexpr int kSpinLimit = 1 << 21;     // polls of a barrier before it gives up

struct TridJob {
    const double* A;                   // n x n, column-major (ld lda), both triangles
    int n, lda, G, R;                  // order, leading dim, workgroups, LDS rows per workgroup
    double *d, *e, *tau, *V, *scale;   // outputs (scaled by *scale)
    double* xbuf;                      // exchange area (xbuf_doubles)
    int* counter;                      // barrier counter (zero at launch)
    int* status;                       // set to 1 if a barrier gave up
};

// Wavefront reductions on DPP lane moves (no LDS round trips): within
// rows of 16 lanes by quad permutations and row mirrors, across rows by the
// row broadcasts of lanes 15 and 31, so that lane 63 holds the result, which
// every lane then reads.  Lanes a DPP move has no source for contribute 0
// (the identity of both reductions below, since max is taken of |x| >= 0 or
// of values whose identity the caller supplies as 0).
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ inline double lane63(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ inline double wave_sum(double x) {
    x += dpp_move<0xB1, 0xF>(x);    // quad_perm [1,0,3,2]
    x += dpp_move<0x4E, 0xF>(x);    // quad_perm [2,3,0,1]
    x += dpp_move<0x141, 0xF>(x);   // row_half_mirror
    x += dpp_move<0x140, 0xF>(x);   // row_mirror: every lane holds its row's sum
    x += dpp_move<0x142, 0xA>(x);   // row_bcast:15 into rows 1, 3
    x += dpp_move<0x143, 0xC>(x);   // row_bcast:31 into rows 2, 3
    return lane63(x);
}
// maximum of values >= 0
__device__ inline double wave_max(double x) {
    x = fmax(x, dpp_move<0xB1, 0xF>(x));
    x = fmax(x, dpp_move<0x4E, 0xF>(x));
    x = fmax(x, dpp_move<0x141, 0xF>(x));
    x = fmax(x, dpp_move<0x140, 0xF>(x));
    x = fmax(x, dpp_move<0x142, 0xA>(x));
    x = fmax(x, dpp_move<0x143, 0xC>(x));
    return lane63(x);
}
// Sum (or max) over the workgroup of NW waves, in a fixed order; every
// thread gets it.
template <int NW>
__device__ double block_sum(double x, double* red) {
    x = wave_sum(x);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += red[i];
    __syncthreads();
    return s;
}
template <int NW>
__device__ double block_max(double x, double* red) {
    x = wave_max(x);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s = fmax(s, red[i]);
    __syncthreads();
    return s;
}

// Values exchanged between the workgroups of a job are written and read
// with relaxed agent-scope atomic accesses, which bypass the caches that are
// not coherent across compute units, so the barrier needs no cache-wide
// write-back or invalidation: each wave waits until its stores have
// completed, then one thread per workgroup adds to the job's counter and
// polls it.  The poll is bounded: after kSpinLimit polls the workgroup
// records the failure and stops waiting at this and every later barrier, so
// the launch always ends.
__device__ inline void st_x(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_x(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ void job_barrier(int* counter, int& epoch, int G, int* failed) {
    ++epoch;
    __builtin_amdgcn_s_waitcnt(0);   // this wave's exchange stores have completed
    __syncthreads();
    if (threadIdx.x == 0 && !*failed) {
        __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int target = epoch * G;
        int polls = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++polls > kSpinLimit) {
                *failed = 1;
                break;
            }
        }
    }
    __syncthreads();
}

// Accesses to a job's exchange area.  Every column writes its own region
// (row and p slices at fresh offsets, each region starting on a 128-byte
// line), so no cache line of the area is read before it is written.  Once
// the workgroups have found that they all run on one XCD (same XCC_ID
// register), plain loads and stores suffice: stores reach the XCD's L2
// before the barrier and the readers' L1 never holds a line of a region
// written later.  Otherwise the agent-scope accesses above are used.
struct Xchg {
    double* base;
    bool local;
    __device__ void st(int64_t idx, double v) const {
        if (local) base[idx] = v;
        else st_x(base + idx, v);
    }
    __device__ double ld(int64_t idx) const { return local ? base[idx] : ld_x(base + idx); }
};
constexpr int kSlots = 2;   // n <= kSlots * kTriThreads: entries j = tid + kTriThreads s per thread

// Step 1.  bmap[b] = (job, rank) of workgroup b; job < 0: idle workgroup.
// Dynamic LDS: R rows of n, v and w of the last two columns (2 x 2 n), the
// reduction scratch.  Thread t owns the entries j = t + kTriThreads q of the
// column vectors (the column, v, p, w), kept in registers.  Per column k:
// (a) the Householder vector from the column (every workgroup; its norm and
// the two leading entries come out of one block reduction); (b) one pass
// over the own rows i > k that applies the pending update of column k-1 and
// forms p_i = tau (row_i . v); the owner of row k+1 publishes it; (c) the
// barrier; (d) p and row k+1 are loaded together, w = p - (tau/2)(p.v) v
// (second block reduction) becomes the pending update and row k+1 with it
// the next column.  Block reductions alternate between two scratch halves,
// so each costs one workgroup barrier.
__device__ inline double block_sum_x(double x, double* red, int& par) {
    x = wave_sum(x);
    double* r = red + par * kTriWaves;
    if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kTriWaves; ++i) s += r[i];
    par ^= 1;
    return s;
}
__global__ __launch_bounds__(kTriThreads) void tridiag_kernel(const TridJob* __restrict__ jobs,
                                                               const int2* __restrict__ bmap) {
    const int2 bm = bmap[blockIdx.x];
    if (bm.x < 0) return;
    const TridJob J = jobs[bm.x];
    const int g = bm.y, G = J.G, n = J.n;
    extern __shared__ double sm[];
    double* rows = sm;
    double* vb = rows + (size_t)J.R * n;   // v of columns k (vb + (k & 1) n)
    double* wb = vb + 2 * (size_t)n;       // w of columns k (wb + (k & 1) n)
    double* red = wb + 2 * (size_t)n;      // 2 x kTriWaves
    double* slot = red + 2 * kTriWaves;    // the column's diagonal entry and alpha
    __shared__ int failed;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) failed = 0;
    int epoch = 0, par = 0;
    const int nloc = g < n ? (n - g + G - 1) / G : 0;   // rows i = g + r G
    // exchange area: G maxima, G XCC ids, then per column k the published
    // row k+1 (npad) and the p slices (npad)
    const int64_t npad = (n + 15) & ~15;
    const int64_t oR = (2 * G + 15) & ~15, oP = oR + (int64_t)n * npad;
    Xchg X;
    X.base = J.xbuf;
    X.local = false;

    double mx = 0.0;
    for (int r = 0; r < nloc; ++r) {
        const int i = g + r * G;
        for (int j = tid; j < n; j += kTriThreads) {
            const double a = J.A[j + (int64_t)i * J.lda];   // row i = column i
            rows[(size_t)r * n + j] = a;
            mx = fmax(mx, fabs(a));
        }
    }
    mx = block_max<kTriWaves>(mx, red);
    if (tid == 0) {
        unsigned xcc;
        __asm__ volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
        X.st(g, mx);
        X.st(G + g, (double)xcc);
    }
    job_barrier(J.counter, epoch, G, &failed);
    double gm = 0.0, other = 0.0;
    const double x0 = X.ld(G);
    for (int t = tid; t < G; t += kTriThreads) {
        gm = fmax(gm, X.ld(t));
        other = fmax(other, X.ld(G + t) != x0 ? 1.0 : 0.0);
    }
    gm = block_max<kTriWaves>(gm, red);
    X.local = block_max<kTriWaves>(other, red) == 0.0;   // every workgroup of the job on one XCD
    const double sc = (gm > 0.0 && isfinite(gm)) ? ldexp(1.0, -ilogb(gm)) : 1.0;
    if (g == 0 && tid == 0) *J.scale = sc;
    for (int r = 0; r < nloc; ++r)
        for (int j = tid; j < n; j += kTriThreads) rows[(size_t)r * n + j] *= sc;
    // the pending update of column -1 is zero
    for (int j = tid; j < n; j += kTriThreads) {
        vb[n + j] = 0.0;
        wb[n + j] = 0.0;
    }
    double col[kSlots], vr[kSlots];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < kSlots; ++q) {
        const int j = tid + q * kTriThreads;
        col[q] = j < n ? J.A[j] * sc : 0.0;   // column 0
        if (j == 0) slot[0] = col[q];
        if (j == 1) slot[1] = col[q];
        if (j >= 2 && j < n) part += col[q] * col[q];
    }
    double xn2 = block_sum_x(part, red, par);
    if (n == 1 && g == 0 && tid == 0) J.d[0] = slot[0];

    for (int k = 0; k + 1 < n; ++k) {
        // (a) Householder vector of column k
        const double dk = slot[0], alpha = slot[1];
        double tau = 0.0, beta = alpha, scal = 0.0;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        double* v = vb + (size_t)(k & 1) * n;
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
            const int j = tid + q * kTriThreads;
            vr[q] = 0.0;
            if (j > k && j < n) {
                vr[q] = j == k + 1 ? 1.0 : col[q] * scal;
                v[j] = vr[q];
                if (g == 0) J.V[(size_t)k * n + j] = vr[q];
            }
        }
        if (g == 0 && tid == 0) {
            J.d[k] = dk;
            J.e[k] = beta;
            J.tau[k] = tau;
        }
        __syncthreads();
        // (b) own rows i > k, one per wave at a time
        const double* vp = vb + (size_t)((k + 1) & 1) * n;   // v, w of column k-1
        const double* wp = wb + (size_t)((k + 1) & 1) * n;
        const int64_t pofs = oP + k * npad, rofs = oR + k * npad;
        const int r0 = k + 1 <= g ? 0 : (k + 1 - g + G - 1) / G;
        for (int r = r0 + wave; r < nloc; r += kTriWaves) {
            const int i = g + r * G;
            double* row = rows + (size_t)r * n;
            const double vpi = vp[i], wpi = wp[i];
            const bool pub = i == k + 1;
            double acc = 0.0;
#pragma unroll 4
            for (int j = k + 1 + lane; j < n; j += 64) {
                const double a = row[j] - vpi * wp[j] - wpi * vp[j];
                row[j] = a;
                acc += a * v[j];
                if (pub) X.st(rofs + j, a);
            }
            acc = wave_sum(acc);
            if (lane == 0) X.st(pofs + i, tau * acc);
        }
        // (c)
        job_barrier(J.counter, epoch, G, &failed);
        // (d) p and row k+1, loaded together
        double pr[kSlots], rr[kSlots];
        const double p1 = X.ld(pofs + k + 1);
        part = 0.0;
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
            const int j = tid + q * kTriThreads;
            pr[q] = rr[q] = 0.0;
            if (j > k && j < n) {
                pr[q] = X.ld(pofs + j);
                rr[q] = X.ld(rofs + j);
            }
            part += pr[q] * vr[q];
        }
        const double c2 = 0.5 * tau * block_sum_x(part, red, par);
        const double w1 = p1 - c2;   // w of entry k+1 (v's entry there is 1)
        double* w = wb + (size_t)(k & 1) * n;
        part = 0.0;
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
            const int j = tid + q * kTriThreads;
            if (j > k && j < n) {
                const double wj = pr[q] - c2 * vr[q];
                w[j] = wj;
                const double c = rr[q] - vr[q] * w1 - wj;   // row k+1 with the update of column k
                col[q] = c;
                if (j == k + 1) slot[0] = c;
                if (j == k + 2) slot[1] = c;
                if (j >= k + 3) part += c * c;
            }
        }
        xn2 = block_sum_x(part, red, par);
        if (k + 2 == n && g == 0 && tid == 0) J.d[n - 1] = slot[0];
    }
    __syncthreads();
    if (tid == 0 && failed) *J.status = 1;
}

struct BisJob {
    const double *d, *e, *scale;
    double* w;      // n eigenvalues, ascending, unscaled
    int n;
};

// Step 2.  bmap[b] = (job, first index); wave q of the workgroup finds the
// eigenvalue of index first + q (ascending).  Dynamic LDS: d and e^2.
__global__ __launch_bounds__(kEigThreads) void bisect_kernel(const BisJob* __restrict__ jobs,
                                                              const int2* __restrict__ bmap) {
    const int2 bm = bmap[blockIdx.x];
    const BisJob J = jobs[bm.x];
    const int n = J.n;
    extern __shared__ double sm[];
    double* d = sm;
    double* e2 = sm + n;
    __shared__ double red[kEigWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double lo = INFINITY, hi = -INFINITY, em = 0.0;
    for (int i = tid; i < n; i += kEigThreads) {
        const double di = J.d[i];
        const double el = i > 0 ? fabs(J.e[i - 1]) : 0.0, er = i + 1 < n ? fabs(J.e[i]) : 0.0;
        d[i] = di;
        e2[i] = er * er;   // e2[i] couples i and i+1
        lo = fmin(lo, di - el - er);
        hi = fmax(hi, di + el + er);
        em = fmax(em, er * er);
    }
    lo = -block_max<kEigWaves>(-lo, red);
    hi = block_max<kEigWaves>(hi, red);
    em = block_max<kEigWaves>(em, red);
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double pivmin = DBL_MIN * fmax(1.0, em);
    const double eps = DBL_EPSILON;
    lo -= 2.0 * eps * tnorm * n + pivmin;
    hi += 2.0 * eps * tnorm * n + pivmin;
    const int j = bm.y + wave;
    if (j >= n) return;   // no block-wide synchronisation below
    if (tnorm == 0.0) {   // T = 0
        if (lane == 0) J.w[j] = 0.0;
        return;
    }
    double a = lo, b = hi;
    for (int pass = 0; pass < 64; ++pass) {
        const double x = a + (b - a) * (double)(lane + 1) / 65.0;
        int cnt = 0;
        double q = d[0] - x;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
        for (int i = 1; i < n; ++i) {
            // e2 / q with the hardware reciprocal and one Newton step
            // (full precision in two fused operations instead of a
            // division's sequence)
            const double r0 = __builtin_amdgcn_rcp(q);
            const double r1 = fma(r0, fma(-q, r0, 1.0), r0);
            q = (d[i] - x) - e2[i - 1] * r1;
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += q < 0.0;
        }
        const unsigned long long above = __ballot(cnt > j);
        const int m = above ? __ffsll((long long)above) - 1 : 64;
        const double xm1 = __shfl(x, m > 0 ? m - 1 : 0, 64);
        const double xm = __shfl(x, m < 64 ? m : 63, 64);
        const double na = m > 0 ? xm1 : a, nb = m < 64 ? xm : b;
        const bool stuck = na == a && nb == b;
        a = na;
        b = nb;
        if (stuck || b - a <= fmax(2.0 * eps * fmax(fabs(a), fabs(b)), eps * tnorm)) break;
    }
    if (lane == 0) J.w[j] = 0.5 * (a + b) / *J.scale;
}

// Inverse iteration solves per eigenvector: from a random start, the first
// solve leaves an error of about |lambda error| / gap, the second one at
// rounding level (eigenvalues from the multisection are accurate to
// 2 eps ||T||).
constexpr int kInvIters = 2;

struct VecJob {
    const double *d, *e, *scale, *w;   // w: eigenvalues ascending, unscaled
    double* Zt;                        // n x kv eigenvectors of T (column j: j-th largest)
    double* work;                      // 5 n per cluster slot
    int n, kv;
};
struct VecCluster {
    int job, first, count, pad;        // eigenvalue ranks first .. first+count-1 (descending)
    int64_t woff;                      // offset of its 5 n doubles of LU work space
};

__device__ inline double start_entry(int i, int m) {
    // fixed pseudo-random start vector entries in (-1, 1) (a 32-bit integer hash)
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ ((uint32_t)m + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return ((double)h + 0.5) / 2147483648.0 - 1.0;
}

// Step 3: one wavefront per cluster.  Lane 0 runs the recurrences of the
// LU factorisation and the solves on LDS arrays, carrying the values each
// step depends on in registers; the whole wave does the vector operations.
// Dynamic LDS: 8 n doubles.
__global__ __launch_bounds__(64) void tdvec_kernel(const VecJob* __restrict__ jobs,
                                                    const VecCluster* __restrict__ clusters) {
    const VecCluster C = clusters[blockIdx.x];
    const VecJob J = jobs[C.job];
    const int n = J.n, lane = threadIdx.x;
    extern __shared__ double sm[];
    double *d = sm, *e = sm + n, *dl = sm + 2 * n, *du = sm + 3 * n, *du2 = sm + 4 * n, *rdd = sm + 5 * n,
           *piv = sm + 6 * n, *z = sm + 7 * n;
    double tl = 0.0;
    for (int i = lane; i < n; i += 64) {
        d[i] = J.d[i];
        e[i] = i + 1 < n ? J.e[i] : 0.0;
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64)
        tl = fmax(tl, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + fabs(e[i]));
    const double tnorm = wave_max(tl);
    const double small = DBL_EPSILON * tnorm;
    const double sc = *J.scale;
    for (int m = 0; m < C.count; ++m) {
        const int jr = C.first + m;                 // rank (descending)
        const double lam = J.w[n - 1 - jr] * sc;    // scaled eigenvalue
        double* zo = J.Zt + (size_t)jr * n;
        if (n == 1 || tnorm == 0.0) {               // T = 0: the unit vectors
            for (int i = lane; i < n; i += 64) zo[i] = i == jr ? 1.0 : 0.0;
            __syncthreads();
            continue;
        }
        {
            // first the twisted factorisation (as in twist_kernel, both
            // recurrences on lane 0, dl and du holding D+ and D-), then the
            // cluster's earlier vectors projected out; unless little is left
            // (the value degenerate with an earlier one), that is the vector
            const double pv = DBL_MIN * fmax(1.0, tnorm * tnorm) / DBL_EPSILON;
            auto guard = [&](double q) { return fabs(q) < pv ? (q < 0.0 ? -pv : pv) : q; };
            auto rcp = [&](double q) {
                const double r0 = __builtin_amdgcn_rcp(q);
                return fma(r0, fma(-q, r0, 1.0), r0);
            };
            if (lane == 0) {
                double q = guard(d[0] - lam);
                dl[0] = q;
                for (int i = 1; i < n; ++i) {
                    q = guard((d[i] - lam) - e[i - 1] * e[i - 1] * rcp(q));
                    dl[i] = q;
                }
                q = guard(d[n - 1] - lam);
                du[n - 1] = q;
                for (int i = n - 2; i >= 0; --i) {
                    q = guard((d[i] - lam) - e[i] * e[i] * rcp(q));
                    du[i] = q;
                }
            }
            __syncthreads();
            double bv = INFINITY;
            int bi = n;
            for (int i = lane; i < n; i += 64) {
                const double gv = fabs(dl[i] + du[i] - (d[i] - lam));
                if (gv < bv) {
                    bv = gv;
                    bi = i;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ov < bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            const int r = bi;
            for (int i = lane; i < n; i += 64) z[i] = i < r ? -e[i] / dl[i] : (i > r ? -e[i - 1] / du[i] : 1.0);
            __syncthreads();
            if (lane == 0) {
                double c = 1.0;
                for (int i = r - 1; i >= 0; --i) {
                    c *= z[i];
                    z[i] = c;
                }
                c = 1.0;
                for (int i = r + 1; i < n; ++i) {
                    c *= z[i];
                    z[i] = c;
                }
            }
            __syncthreads();
            double part = 0.0;
            for (int i = lane; i < n; i += 64) part += z[i] * z[i];
            double inv = 1.0 / sqrt(wave_sum(part));
            for (int i = lane; i < n; i += 64) z[i] *= inv;
            for (int q = 0; q < m; ++q) {
                const double* y = J.Zt + (size_t)(C.first + q) * n;
                double pq = 0.0;
                for (int i = lane; i < n; i += 64) pq += y[i] * z[i];
                const double dot = wave_sum(pq);
                for (int i = lane; i < n; i += 64) z[i] -= dot * y[i];
            }
            part = 0.0;
            for (int i = lane; i < n; i += 64) part += z[i] * z[i];
            const double left = wave_sum(part);
            if (left >= 0.25) {
                inv = 1.0 / sqrt(left);
                for (int i = lane; i < n; i += 64) zo[i] = z[i] * inv;
                __syncthreads();   // later members of the cluster read this vector
                continue;
            }
            __syncthreads();
        }
        if (lane == 0) {
            // LU with partial pivoting of T - lam I (LAPACK's tridiagonal
            // scheme; row interchanges recorded in piv, tiny pivots raised
            // to eps ||T||, reciprocals of the pivots kept).  The entries of
            // the next step are loaded one step ahead.
            double cd = d[0] - lam, cu = e[0];
            double sub = e[0], dnx = d[1], enx = n > 2 ? e[1] : 0.0;
            for (int i = 0; i + 1 < n; ++i) {
                const double s0 = sub;
                double nd = dnx - lam, nu = enx;
                sub = enx;
                dnx = i + 2 < n ? d[i + 2] : 0.0;
                enx = i + 3 < n ? e[i + 2] : 0.0;
                if (fabs(cd) >= fabs(s0)) {
                    if (fabs(cd) < small) cd = cd < 0.0 ? -small : small;
                    const double r0 = __builtin_amdgcn_rcp(cd);
                    const double r = fma(r0, fma(-cd, r0, 1.0), r0);
                    const double f = s0 * r;
                    dl[i] = f;
                    du[i] = cu;
                    du2[i] = 0.0;
                    rdd[i] = r;
                    piv[i] = 0.0;
                    nd -= f * cu;
                } else {
                    const double r0 = __builtin_amdgcn_rcp(s0);
                    const double r = fma(r0, fma(-s0, r0, 1.0), r0);
                    const double f = cd * r;
                    dl[i] = f;
                    rdd[i] = r;
                    du[i] = nd;
                    du2[i] = nu;
                    piv[i] = 1.0;
                    nd = cu - f * nd;
                    nu = -f * nu;
                }
                cd = nd;
                cu = nu;
            }
            if (fabs(cd) < small) cd = cd < 0.0 ? -small : small;
            rdd[n - 1] = 1.0 / cd;
        }
        for (int i = lane; i < n; i += 64) z[i] = start_entry(i, jr);
        __syncthreads();
        for (int it = 0; it < kInvIters; ++it) {
            if (lane == 0) {
                // L U y = P z in place: forward with the interchanges ...
                double zi = z[0];
                double zn = z[1], pv = piv[0], f = dl[0];
                for (int i = 0; i + 1 < n; ++i) {
                    const double zn0 = zn, pv0 = pv, f0 = f;
                    if (i + 2 < n) {
                        zn = z[i + 2];
                        pv = piv[i + 1];
                        f = dl[i + 1];
                    }
                    if (pv0 == 0.0) {
                        z[i] = zi;
                        zi = zn0 - f0 * zi;
                    } else {
                        z[i] = zn0;
                        zi = zi - f0 * zn0;
                    }
                }
                // ... then back substitution
                double z1 = zi * rdd[n - 1];
                z[n - 1] = z1;
                double z2 = 0.0;
                double zc_in = z[n - 2], u1 = du[n - 2], u2 = du2[n - 2], rr = rdd[n - 2];
                for (int i = n - 2; i >= 0; --i) {
                    const double a0 = zc_in, a1 = u1, a2 = u2, a3 = rr;
                    if (i > 0) {
                        zc_in = z[i - 1];
                        u1 = du[i - 1];
                        u2 = du2[i - 1];
                        rr = rdd[i - 1];
                    }
                    const double zc = (a0 - a1 * z1 - a2 * z2) * a3;
                    z[i] = zc;
                    z2 = z1;
                    z1 = zc;
                }
            }
            __syncthreads();
            // against the cluster's earlier vectors
            for (int q = 0; q < m; ++q) {
                const double* y = J.Zt + (size_t)(C.first + q) * n;
                double part = 0.0;
                for (int i = lane; i < n; i += 64) part += y[i] * z[i];
                const double dot = wave_sum(part);
                for (int i = lane; i < n; i += 64) z[i] -= dot * y[i];
            }
            double mx = 0.0;
            for (int i = lane; i < n; i += 64) mx = fmax(mx, fabs(z[i]));
            mx = wave_max(mx);
            const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
            double part = 0.0;
            for (int i = lane; i < n; i += 64) {
                const double v = z[i] * inv;
                z[i] = v;
                part += v * v;
            }
            const double r = 1.0 / sqrt(wave_sum(part));
            for (int i = lane; i < n; i += 64) z[i] *= r;
            __syncthreads();
        }
        for (int i = lane; i < n; i += 64) zo[i] = z[i];
        __syncthreads();   // later members of the cluster read this vector
    }
}

// Step 3 for an eigenvalue apart from the others (a cluster of one): the
// eigenvector straight from the twisted factorisation of T - lam I.  Wave 0
// runs the top-down recurrence D+_i = (d_i - lam) - e_{i-1}^2 / D+_{i-1},
// wave 1 the bottom-up one D-_i = (d_i - lam) - e_i^2 / D-_{i+1} at the same
// time; the twist r minimises |gamma_i| = |D+_i + D-_i - (d_i - lam)| (ties:
// the lower index); then z_r = 1, z_i = -e_i z_{i+1} / D+_i above r and
// z_i = -e_{i-1} z_{i-1} / D-_i below it, normalised.  Its residual is
// |gamma_r| / ||z||, which an eigenvalue accurate to 2 eps ||T|| keeps at
// rounding level (no iteration).  Dynamic LDS: d, e, D+, D-, z (5 n).
__global__ __launch_bounds__(128) void twist_kernel(const VecJob* __restrict__ jobs,
                                                     const VecCluster* __restrict__ clusters) {
    const VecCluster C = clusters[blockIdx.x];
    const VecJob J = jobs[C.job];
    const int n = J.n, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    extern __shared__ double sm[];
    double *d = sm, *e = sm + n, *dp = sm + 2 * n, *dm = sm + 3 * n, *z = sm + 4 * n;
    __shared__ double red_v[2];
    __shared__ int red_i[2];
    for (int i = tid; i < n; i += 128) {
        d[i] = J.d[i];
        e[i] = i + 1 < n ? J.e[i] : 0.0;
    }
    __syncthreads();
    double tl = 0.0, em = 0.0;
    for (int i = tid; i < n; i += 128) {
        tl = fmax(tl, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + fabs(e[i]));
        em = fmax(em, e[i] * e[i]);
    }
    tl = wave_max(tl);
    em = wave_max(em);
    if (lane == 0) red_v[wave] = tl;
    __syncthreads();
    const double tnorm = fmax(red_v[0], red_v[1]);
    __syncthreads();
    const int jr = C.first;
    double* zo = J.Zt + (size_t)jr * n;
    if (n == 1 || tnorm == 0.0) {   // T = 0: the unit vectors
        for (int i = tid; i < n; i += 128) zo[i] = i == jr ? 1.0 : 0.0;
        return;
    }
    const double lam = J.w[n - 1 - jr] * *J.scale;
    // pivots below this are raised to it (keeping the sign): never zero
    const double piv = DBL_MIN * fmax(1.0, em) / DBL_EPSILON;
    auto guard = [&](double q) { return fabs(q) < piv ? (q < 0.0 ? -piv : piv) : q; };
    auto rcp = [&](double q) {
        const double r0 = __builtin_amdgcn_rcp(q);
        return fma(r0, fma(-q, r0, 1.0), r0);
    };
    if (lane == 0 && wave == 0) {
        double q = guard(d[0] - lam);
        dp[0] = q;
        double dn = d[1], ep = e[0];
        for (int i = 1; i < n; ++i) {
            const double a = dn - lam, e2 = ep * ep;
            if (i + 1 < n) {
                dn = d[i + 1];
                ep = e[i];
            }
            q = guard(a - e2 * rcp(q));
            dp[i] = q;
        }
    } else if (lane == 0 && wave == 1) {
        double q = guard(d[n - 1] - lam);
        dm[n - 1] = q;
        double dn = d[n - 2], ep = e[n - 2];
        for (int i = n - 2; i >= 0; --i) {
            const double a = dn - lam, e2 = ep * ep;
            if (i > 0) {
                dn = d[i - 1];
                ep = e[i - 1];
            }
            q = guard(a - e2 * rcp(q));
            dm[i] = q;
        }
    }
    __syncthreads();
    // twist: argmin |gamma| (lowest index on ties)
    double bv = INFINITY;
    int bi = n;
    for (int i = tid; i < n; i += 128) {
        const double g = fabs(dp[i] + dm[i] - (d[i] - lam));
        if (g < bv) {
            bv = g;
            bi = i;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov < bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane == 0) {
        red_v[wave] = bv;
        red_i[wave] = bi;
    }
    __syncthreads();
    const int r = (red_v[1] < red_v[0] || (red_v[1] == red_v[0] && red_i[1] < red_i[0])) ? red_i[1] : red_i[0];
    // ratios in parallel, then the two product chains at once
    for (int i = tid; i < n; i += 128) {
        if (i < r) z[i] = -e[i] / dp[i];
        else if (i > r) z[i] = -e[i - 1] / dm[i];
        else z[i] = 1.0;
    }
    __syncthreads();
    if (lane == 0 && wave == 0) {
        double c = 1.0;
        for (int i = r - 1; i >= 0; --i) {
            c *= z[i];
            z[i] = c;
        }
    } else if (lane == 0 && wave == 1) {
        double c = 1.0;
        for (int i = r + 1; i < n; ++i) {
            c *= z[i];
            z[i] = c;
        }
    }
    __syncthreads();
    double part = 0.0;
    for (int i = tid; i < n; i += 128) part += z[i] * z[i];
    part = wave_sum(part);
    if (lane == 0) red_v[wave] = part;
    __syncthreads();
    const double inv = 1.0 / sqrt(red_v[0] + red_v[1]);
    for (int i = tid; i < n; i += 128) zo[i] = z[i] * inv;
}

struct BackJob {
    const double *V, *tau, *Zt;
    double* Z;      // n x kv, column-major
    int n, kv;
};

// Step 4.  One workgroup per eigenvector (bmap[b] = (job, vector)); thread
// t owns the rows i = t + kBackThreads s.  The reflectors are applied one at
// a time (one block-wide reduction each, its scratch alternating between two
// halves so that one barrier per reflector suffices).  They are streamed
// through LDS in chunks of up to kChunk consecutive reflectors (contiguous
// in V, read as 16-byte pairs): the loads of the next chunk are issued into
// registers before the current chunk is applied, so their latency overlaps
// its work.  Entries a reflector does not store (rows i <= j) are never
// read.  Dynamic LDS: the vector, tau, one chunk.  A cut keeps few vectors
// (one workgroup each, on a fraction of the compute units), so the
// per-reflector latency sets the time: eight waves (0.43 ms for the 65
// vectors of the D = 6, chi = 64 cut) beat four (0.50) and sixteen (0.50).
constexpr int kBackThreads = 512;
constexpr int kBackWaves = kBackThreads / 64;
constexpr int kChunk = 16;        // reflectors per chunk at most
constexpr int kChunkLoads = 8;    // 16-byte loads per thread per chunk at most (the chunk size follows)
__global__ __launch_bounds__(kBackThreads) void backtr_kernel(const BackJob* __restrict__ jobs,
                                                               const int2* __restrict__ bmap, int ch) {
    const int2 bm = bmap[blockIdx.x];
    const BackJob J = jobs[bm.x];
    const int n = J.n, c0 = bm.y;
    extern __shared__ double z[];
    double* taus = z + n;
    double* vb = taus + n;   // the chunk as loaded: V's doubles from index 2 p0 on
    __shared__ double red[2][kBackWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < n; i += kBackThreads) {
        z[i] = J.Zt[(size_t)c0 * n + i];
        taus[i] = J.tau[i];
    }
    const double2* V2 = reinterpret_cast<const double2*>(J.V);
    // chunk with last reflector jb covers reflectors max(jb - kChunk + 1, 0) .. jb,
    // rows jl .. jb of V: doubles [jl n, (jb + 1) n) read as whole 16-byte pairs
    auto chunk_range = [&](int jb, int64_t& p0, int& np) {
        const int jl = max(jb - ch + 1, 0);
        p0 = ((int64_t)jl * n) >> 1;
        np = (int)((((int64_t)(jb + 1) * n + 1) >> 1) - p0);
    };
    double2 rg[kChunkLoads];
    int64_t p0 = 0;
    int np = 0;
    if (n >= 2) {
        chunk_range(n - 2, p0, np);
#pragma unroll
        for (int u = 0; u < kChunkLoads; ++u) {
            const int e = tid + u * kBackThreads;
            rg[u] = e < np ? V2[p0 + e] : make_double2(0.0, 0.0);
        }
    }
    int par = 0;
    for (int jb = n - 2; jb >= 0; jb -= ch) {
        __syncthreads();   // the previous chunk is applied
        chunk_range(jb, p0, np);
        const int64_t base = 2 * p0;   // V index of vb[0]
#pragma unroll
        for (int u = 0; u < kChunkLoads; ++u) {
            const int e = tid + u * kBackThreads;
            if (e < np) reinterpret_cast<double2*>(vb)[e] = rg[u];
        }
        if (jb - ch >= 0) {
            int64_t p1;
            int np1;
            chunk_range(jb - ch, p1, np1);
#pragma unroll
            for (int u = 0; u < kChunkLoads; ++u) {
                const int e = tid + u * kBackThreads;
                rg[u] = e < np1 ? V2[p1 + e] : make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
        const int jl = max(jb - ch + 1, 0);
        for (int j = jb; j >= jl; --j) {
            const double tj = taus[j];
            if (tj == 0.0) continue;
            const double* v = vb + ((int64_t)j * n - base);
            double part = 0.0;
#pragma unroll
            for (int q = 0; q < kSlots * (kTriThreads / kBackThreads); ++q) {
                const int i = tid + q * kBackThreads;
                if (i > j && i < n) part += v[i] * z[i];
            }
            part = wave_sum(part);
            if (lane == 0) red[par][wave] = part;
            __syncthreads();
            double f = 0.0;
#pragma unroll
            for (int q = 0; q < kBackWaves; ++q) f += red[par][q];
            f *= tj;
#pragma unroll
            for (int q = 0; q < kSlots * (kTriThreads / kBackThreads); ++q) {
                const int i = tid + q * kBackThreads;
                if (i > j && i < n) z[i] -= f * v[i];
            }
            par ^= 1;
        }
    }
    __syncthreads();
    for (int i = tid; i < n; i += kBackThreads) J.Z[(size_t)c0 * n + i] = z[i];
}

struct DevInfo {
    int lds = 0, cus = 0;
};
DevInfo dev_info() {
    static std::mutex mu;
    static std::map<int, DevInfo> cache;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    DevInfo di;
    int lds = 0, cus = 0;
    HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    di.lds = std::min(lds, 160 * 1024) - 4096;   // room for the kernels' static shared variables
    di.cus = cus;
    cache[dev] = di;
    return di;
}

// LDS rows per workgroup and workgroups of a job of order n (0, 0 if it
// does not fit the chip's LDS).
void tridiag_shape(int n, const DevInfo& di, int& R, int& G) {
    R = G = 0;
    const int64_t doubles = di.lds / 8 - 4LL * n - 2 * kTriWaves - 2;
    if (n <= 0 || doubles < n) return;
    R = (int)std::min<int64_t>(doubles / n, n);
    G = (n + R - 1) / R;
    // the vector steps' limits: rows per back-transformation thread and the
    // LDS of their blocks of vectors
    if (G > di.cus || n > kSlots * kTriThreads || 8LL * (3 * n + 4) > di.lds) R = G = 0;
}

// Descriptors go to the device through a ring of pinned host memory and an
// asynchronous copy on the caller's stream (no host synchronisation inside a
// move).  A range of the ring is reused once the event recorded after its
// copy has completed.
class PinnedRing {
  public:
    void upload(BufferPtr& dst, const void* src, size_t bytes, hipStream_t s) {
        dst = device_alloc(std::max<size_t>(bytes, 16));
        if (!bytes) return;
        std::lock_guard<std::mutex> lk(mu_);
        const size_t need = (bytes + 255) & ~(size_t)255;
        if (need > kCap) {   // larger than the ring: a synchronous copy
            HIPCHK(hipMemcpy(dst->ptr, src, bytes, hipMemcpyHostToDevice));
            return;
        }
        if (!host_) HIPCHK(hipHostMalloc((void**)&host_, kCap, hipHostMallocDefault));
        if (head_ + need > kCap) head_ = 0;
        // wait for earlier copies out of [head_, head_ + need)
        for (auto it = inflight_.begin(); it != inflight_.end();) {
            if (it->off < head_ + need && head_ < it->off + it->len) {
                HIPCHK(hipEventSynchronize(it->ev));
                free_.push_back(it->ev);
                it = inflight_.erase(it);
            } else {
                ++it;
            }
        }
        std::memcpy(host_ + head_, src, bytes);
        HIPCHK(hipMemcpyAsync(dst->ptr, host_ + head_, bytes, hipMemcpyHostToDevice, s));
        hipEvent_t ev;
        if (free_.empty()) {
            HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        } else {
            ev = free_.back();
            free_.pop_back();
        }
        HIPCHK(hipEventRecord(ev, s));
        inflight_.push_back({head_, need, ev});
        head_ += need;
    }

  private:
    static constexpr size_t kCap = 4 << 20;
    struct Range {
        size_t off, len;
        hipEvent_t ev;
    };
    std::mutex mu_;
    char* host_ = nullptr;
    size_t head_ = 0;
    std::vector<Range> inflight_;
    std::vector<hipEvent_t> free_;
};

void upload_async(BufferPtr& dst, const void* src, size_t bytes, hipStream_t s) {
    static std::mutex mu;
    static std::map<int, PinnedRing*> rings;   // one per device, kept for the process
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    PinnedRing* r;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto& slot = rings[dev];
        if (!slot) slot = new PinnedRing();
        r = slot;
    }
    r->upload(dst, src, bytes, s);
}

// Dynamic LDS limits of the solver's kernels, raised once per device.
void set_lds_limits(const DevInfo& di) {
    static std::mutex mu;
    static std::set<int> done;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (done.count(dev)) return;
    const char* names[] = {"tridiag", "bisect", "backtr", "tdvec", "twist"};
    const void* fns[] = {(const void*)tridiag_kernel, (const void*)bisect_kernel, (const void*)backtr_kernel,
                         (const void*)tdvec_kernel, (const void*)twist_kernel};
    for (int i = 0; i < 5; ++i) {
        const hipError_t e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, di.lds);
        if (e != hipSuccess)
            fail(SYMTEN_E_HIP, std::string("eigh: dynamic LDS limit of the ") + names[i] + " kernel: " +
                                   hipGetErrorString(e));
    }
    done.insert(dev);
}

// Doubles of a job's exchange area: maxima and XCC ids, then two regions
// of n rounded up to 16 doubles per column.
size_t xbuf_doubles(int n, int G) {
    const size_t npad = ((size_t)n + 15) & ~(size_t)15;
    return (((size_t)2 * G + 15) & ~(size_t)15) + 2 * (size_t)n * npad;
}

}  // namespace

struct EighWork {
    std::vector<EighProblem> probs;
    std::vector<BufferPtr> keep;
    std::vector<double*> d, e, tau, V, scale, w;
    int* status = nullptr;               // one per problem
};

bool eigh_fits(int n) {
    int R, G;
    tridiag_shape(n, dev_info(), R, G);
    return G > 0;
}

int eigh_problems(const EighWork& wk) { return (int)wk.probs.size(); }

int eigh_max_order() {
    const DevInfo di = dev_info();
    int lo = 1, hi = 1 << 16;   // largest n that fits (fits is monotone in n)
    int R, G;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        tridiag_shape(mid, di, R, G);
        if (G > 0) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

std::shared_ptr<EighWork> eigh_values(const std::vector<EighProblem>& probs, hipStream_t s) {
    auto wk = std::make_shared<EighWork>();
    wk->probs = probs;
    const int np = (int)probs.size();
    if (np == 0) return wk;
    const DevInfo di = dev_info();
    std::vector<int> Rs(np), Gs(np);
    size_t doubles = 0;
    int nmax = 0;
    for (int p = 0; p < np; ++p) {
        const int n = probs[p].n;
        if (n < 1 || probs[p].lda < n || !probs[p].A || !probs[p].w) fail(SYMTEN_E_INVAL, "eigh: bad problem");
        tridiag_shape(n, di, Rs[p], Gs[p]);
        if (Gs[p] == 0) fail(SYMTEN_E_CAPACITY, "eigh: matrix of order " + std::to_string(n) + " exceeds the LDS of the chip");
        doubles += 3 * (size_t)n + (size_t)n * n + 1 + xbuf_doubles(n, Gs[p]);
        nmax = std::max(nmax, n);
    }
    BufferPtr buf = device_alloc(8 * doubles + 8 * (size_t)np * 2);
    BufferPtr ibuf = device_alloc(sizeof(int) * 2 * (size_t)np);
    launch_fill_zero(ibuf->ptr, sizeof(int) * 2 * (int64_t)np, s);
    wk->keep = {buf, ibuf};
    int* counters = (int*)ibuf->ptr;
    wk->status = counters + np;
    std::vector<TridJob> tj(np);
    // the exchange areas first (each a multiple of 16 doubles, so each
    // starts on a 128-byte line of the pool's aligned block), then the rest
    double* q = (double*)buf->ptr;
    for (int p = 0; p < np; ++p) {
        tj[p].xbuf = q;
        q += xbuf_doubles(probs[p].n, Gs[p]);
    }
    for (int p = 0; p < np; ++p) {
        const int n = probs[p].n;
        TridJob& J = tj[p];
        J.A = probs[p].A;
        J.n = n;
        J.lda = probs[p].lda;
        J.G = Gs[p];
        J.R = Rs[p];
        J.d = q; q += n;
        J.e = q; q += n;
        J.tau = q; q += n;
        J.V = q; q += (size_t)n * n;
        J.scale = q; q += 1;
        J.counter = counters + p;
        J.status = probs[p].status ? probs[p].status : wk->status + p;
        wk->d.push_back(J.d);
        wk->e.push_back(J.e);
        wk->tau.push_back(J.tau);
        wk->V.push_back(J.V);
        wk->scale.push_back(J.scale);
        wk->w.push_back(probs[p].w);
    }
    // ---- launches of step 1: jobs by size, packed into launches of at most
    // one workgroup per compute unit; a job that fits one XCD (cus / 8
    // workgroups) takes blocks b = x (mod 8) of one XCD x
    std::vector<int> order(np);
    for (int p = 0; p < np; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return Gs[a] > Gs[b]; });
    const int per_xcd = std::max(1, di.cus / 8);
    std::vector<std::vector<int>> launches;
    {
        std::vector<int> cur;
        int used = 0;
        for (int p : order) {
            if (used + Gs[p] > di.cus) {
                launches.push_back(cur);
                cur.clear();
                used = 0;
            }
            cur.push_back(p);
            used += Gs[p];
        }
        if (!cur.empty()) launches.push_back(cur);
    }
    const size_t lds_bytes = (size_t)di.lds;
    set_lds_limits(di);
    std::vector<BufferPtr> descs;
    for (auto& L : launches) {
        // slots per XCD: slot t of XCD x is block x + 8 t
        std::vector<std::vector<int2>> xcd(8);
        std::vector<int2> spill;
        for (int p : L) {
            int best = -1;
            if (Gs[p] <= per_xcd)
                for (int x = 0; x < 8; ++x)
                    if ((int)xcd[x].size() + Gs[p] <= per_xcd && (best < 0 || xcd[x].size() < xcd[best].size()))
                        best = x;
            for (int r = 0; r < Gs[p]; ++r) {
                if (best >= 0) xcd[best].push_back(make_int2(p, r));
                else spill.push_back(make_int2(p, r));
            }
        }
        for (auto& sp : spill) {   // jobs wider than an XCD: the emptiest XCDs first
            int x = 0;
            for (int y = 1; y < 8; ++y)
                if (xcd[y].size() < xcd[x].size()) x = y;
            xcd[x].push_back(sp);
        }
        size_t depth = 0;
        for (auto& v : xcd) depth = std::max(depth, v.size());
        std::vector<int2> bmap(8 * depth, make_int2(-1, 0));
        for (int x = 0; x < 8; ++x)
            for (size_t t = 0; t < xcd[x].size(); ++t) bmap[x + 8 * t] = xcd[x][t];
        // the job descriptors and the block map in one upload
        const size_t jb = sizeof(TridJob) * np, mb = sizeof(int2) * bmap.size();
        std::vector<char> host(jb + mb);
        std::memcpy(host.data(), tj.data(), jb);
        std::memcpy(host.data() + jb, bmap.data(), mb);
        BufferPtr db;
        upload_async(db, host.data(), host.size(), s);
        descs.push_back(db);
        const TridJob* djobs = (const TridJob*)db->ptr;
        const int2* dmap = (const int2*)((const char*)db->ptr + jb);
        void* args[] = {(void*)&djobs, (void*)&dmap};
        int64_t flops = 0;   // Householder tridiagonalisation: 4/3 n^3 (FP64)
        for (int p : L) flops += 4 * (int64_t)probs[p].n * probs[p].n * probs[p].n / 3;
        profile_launch("eigh_tridiag", flops, flops, 0, s, [&] {
            HIPCHK(hipLaunchCooperativeKernel((const void*)tridiag_kernel, dim3((unsigned)bmap.size()),
                                              dim3(kTriThreads), args, (unsigned)lds_bytes, s));
        });
    }
    // ---- step 2: one wave per eigenvalue, four per workgroup
    {
        std::vector<BisJob> bj(np);
        std::vector<int2> bmap;
        for (int p = 0; p < np; ++p) {
            bj[p] = BisJob{wk->d[p], wk->e[p], wk->scale[p], probs[p].w, probs[p].n};
            for (int j = 0; j < probs[p].n; j += kEigWaves) bmap.push_back(make_int2(p, j));
        }
        const size_t jb = sizeof(BisJob) * np, mb = sizeof(int2) * bmap.size();
        std::vector<char> host(jb + mb);
        std::memcpy(host.data(), bj.data(), jb);
        std::memcpy(host.data() + jb, bmap.data(), mb);
        BufferPtr db;
        upload_async(db, host.data(), host.size(), s);
        descs.push_back(db);
        const size_t lb = 16 * (size_t)nmax;
        if (lb > lds_bytes) fail(SYMTEN_E_CAPACITY, "eigh: tridiagonal matrix exceeds LDS");
        profile_launch("eigh_bisect", 0, 0, 0, s, [&] {
            hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)bmap.size()), dim3(kEigThreads), lb, s,
                               (const BisJob*)db->ptr, (const int2*)((const char*)db->ptr + jb));
            HIPCHK(hipGetLastError());
        });
    }
    for (auto& b : descs) wk->keep.push_back(b);
    return wk;
}

void eigh_status(const EighWork& wk, hipStream_t s) {
    const int np = (int)wk.probs.size();
    if (np == 0) return;
    std::vector<int> st(np);
    HIPCHK(hipMemcpyAsync(st.data(), wk.status, sizeof(int) * np, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int v : st)
        if (v) fail(SYMTEN_E_HIP, "eigh: the workgroups of a tridiagonalisation did not meet at a barrier");
}

void eigh_vectors(EighWork& wk, const std::vector<int>& kv, const std::vector<double*>& Z,
                  const std::vector<const double*>& w_host, hipStream_t s) {
    const int np = (int)wk.probs.size();
    if ((int)kv.size() != np || (int)Z.size() != np || (int)w_host.size() != np)
        fail(SYMTEN_E_INVAL, "eigh_vectors: one entry per problem");
    // clusters of close eigenvalues (descending), from the host copy of w
    std::vector<VecCluster> cl;
    size_t ztot = 0;
    for (int p = 0; p < np; ++p) {
        const int n = wk.probs[p].n, k = kv[p];
        if (k < 0 || k > n) fail(SYMTEN_E_INVAL, "eigh_vectors: vector count out of range");
        if (k == 0) continue;
        const double* w = w_host[p];
        const double tn = std::max(std::fabs(w[0]), std::fabs(w[n - 1]));
        const double ortol = 1e-3 * tn;
        int j = 0;
        while (j < k) {
            int c = 1;
            while (j + c < k && w[n - 1 - (j + c - 1)] - w[n - 1 - (j + c)] <= ortol) ++c;
            cl.push_back(VecCluster{p, j, c, 0});
            j += c;
        }
        ztot += (size_t)n * k;
    }
    if (cl.empty()) return;
    std::stable_partition(cl.begin(), cl.end(), [](const VecCluster& c) { return c.count == 1; });
    int n_single = 0;
    for (auto& c : cl) n_single += c.count == 1;
    size_t worktot = 0;
    for (auto& c : cl) {
        c.woff = (int64_t)worktot;
        worktot += 5 * (size_t)wk.probs[c.job].n;
    }
    BufferPtr zt = device_alloc(8 * ztot);
    BufferPtr work = device_alloc(8 * worktot);
    std::vector<VecJob> vj(np);
    std::vector<BackJob> bj(np);
    std::vector<int2> bmap;
    size_t zo = 0;
    for (int p = 0; p < np; ++p) {
        const int n = wk.probs[p].n;
        vj[p] = VecJob{wk.d[p], wk.e[p], wk.scale[p], wk.w[p], (double*)zt->ptr + zo, (double*)work->ptr, n, kv[p]};
        bj[p] = BackJob{wk.V[p], wk.tau[p], (double*)zt->ptr + zo, Z[p], n, kv[p]};
        for (int c = 0; c < kv[p]; ++c) bmap.push_back(make_int2(p, c));
        zo += (size_t)n * kv[p];
    }
    const size_t b1 = sizeof(VecJob) * np, b2 = sizeof(VecCluster) * cl.size(), b3 = sizeof(BackJob) * np,
                 b4 = sizeof(int2) * bmap.size();
    std::vector<char> host(b1 + b2 + b3 + b4);
    std::memcpy(host.data(), vj.data(), b1);
    std::memcpy(host.data() + b1, cl.data(), b2);
    std::memcpy(host.data() + b1 + b2, bj.data(), b3);
    std::memcpy(host.data() + b1 + b2 + b3, bmap.data(), b4);
    BufferPtr db;
    upload_async(db, host.data(), host.size(), s);
    const char* base = (const char*)db->ptr;
    int nmax = 0;
    for (auto& pr : wk.probs) nmax = std::max(nmax, pr.n);
    const DevInfo di = dev_info();
    set_lds_limits(di);
    const size_t lv = 8 * 8 * (size_t)nmax;
    // reflectors per chunk: the registers of a chunk's loads (its doubles,
    // plus one pair at each end) and LDS bound it
    const int ch = (int)std::max<int64_t>(1, std::min<int64_t>(kChunk, (2LL * kChunkLoads * kBackThreads - 4) / nmax));
    const size_t lb = 8 * ((size_t)(ch + 2) * nmax + 4);
    if (lb > (size_t)di.lds || lv > (size_t)di.lds || nmax > kSlots * kTriThreads)
        fail(SYMTEN_E_CAPACITY, "eigh: vectors exceed LDS");
    // clusters of one first in the list (the twisted factorisation), then
    // the rest (inverse iteration with reorthogonalisation)
    const int nsingle = n_single;
    if (nsingle > 0)
        profile_launch("eigh_twist", 0, 0, 0, s, [&] {
            hipLaunchKernelGGL(twist_kernel, dim3((unsigned)nsingle), dim3(128), 8 * 5 * (size_t)nmax, s,
                               (const VecJob*)base, (const VecCluster*)(base + b1));
            HIPCHK(hipGetLastError());
        });
    if ((int)cl.size() > nsingle)
        profile_launch("eigh_tdvec", 0, 0, 0, s, [&] {
            hipLaunchKernelGGL(tdvec_kernel, dim3((unsigned)(cl.size() - nsingle)), dim3(64), lv, s,
                               (const VecJob*)base, (const VecCluster*)(base + b1) + nsingle);
            HIPCHK(hipGetLastError());
        });
    int64_t bflops = 0;   // back-transformation: 2 n^2 per vector
    for (int p = 0; p < np; ++p) bflops += 2 * (int64_t)wk.probs[p].n * wk.probs[p].n * kv[p];
    profile_launch("eigh_backtr", bflops, bflops, 0, s, [&] {
        hipLaunchKernelGGL(backtr_kernel, dim3((unsigned)bmap.size()), dim3(kBackThreads), lb, s,
                           (const BackJob*)(base + b1 + b2), (const int2*)(base + b1 + b2 + b3), ch);
        HIPCHK(hipGetLastError());
    });
    wk.keep.push_back(zt);
    wk.keep.push_back(work);
    wk.keep.push_back(db);
}

}  // namespace symten
