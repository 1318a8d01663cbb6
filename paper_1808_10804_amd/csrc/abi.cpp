// C ABI of libsymten and the CTM move (enlarged corners, halves, FP64
// projectors through rocSOLVER/rocBLAS, renormalisation, normalisation).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <list>
#include <map>
#include <sstream>
#include <exception>
#include <mutex>
#include <system_error>
#include <thread>
#include <numeric>
#include <unordered_map>

#include "internal.hpp"

struct symten_tensor {
    symten::TensorPtr t;
};

namespace symten {

void upload_sync(BufferPtr& buf, const void* host, size_t bytes);
void copy_prefix(const std::vector<CopyTask>& tasks, std::vector<int64_t>& prefix);
void copy_launch_dev(const CopyTask* d_tasks, const int64_t* d_prefix, int ntasks, int64_t npieces,
                     void* const* d_ptrs, bool src_f64, int dst_kind, hipStream_t s);
int choose_tile_cfg(const ContractPlan& p);
void launch_scale_cols(double* X, int ld, int rows, int cols, const double* s, double e, hipStream_t st);
void launch_scale_rows(double* X, int ld, int rows, int cols, const double* s, double e, hipStream_t st);
void launch_eig_to_svd(const double* Z, int NE, const double* w, int voff, int mn, int ru, int rd, bool jw,
                       double* S, double* U, double* V, hipStream_t st);
// zero-padded batches of col-major blocks for the projector factorizations
constexpr int kMaxPadBatch = 32;
struct PadArgs {
    const void* src[kMaxPadBatch];
    int rows[kMaxPadBatch];
    int cols[kMaxPadBatch];
    int count, N;
    bool src_f64;
};
void launch_pad_blocks(const PadArgs& a, double* dst, hipStream_t st);
void launch_jw_build_batched(const double* M, int N, int count, double* J, hipStream_t st);
void launch_nonfinite_guard(double* X, int64_t n, int* flag, hipStream_t st);

namespace {
thread_local std::string g_err;

int set_err(int code, const std::string& m) {
    g_err = m;
    return code;
}

template <class F>
int guard(F&& f) {
    try {
        f();
        return SYMTEN_OK;
    } catch (const Error& e) {
        return set_err(e.code, e.what());
    } catch (const std::bad_alloc&) {
        return set_err(SYMTEN_E_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return set_err(SYMTEN_E_INVAL, e.what());
    } catch (...) {
        return set_err(SYMTEN_E_INVAL, "unknown error");
    }
}

// guard() for entry points that enqueue on `stream`: the library's buffers
// taken and released during the call are ordered on that stream.
template <class F>
int guard_on(void* stream, F&& f) {
    StreamScope scope((hipStream_t)stream);
    try {
        f();
        return SYMTEN_OK;
    } catch (const Error& e) {
        return set_err(e.code, e.what());
    } catch (const std::bad_alloc&) {
        return set_err(SYMTEN_E_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return set_err(SYMTEN_E_INVAL, e.what());
    } catch (...) {
        return set_err(SYMTEN_E_INVAL, "unknown error");
    }
}

Tensor& T(symten_t h) {
    if (!h || !h->t) fail(SYMTEN_E_INVAL, "null tensor handle");
    return *h->t;
}

symten_t wrap(TensorPtr p) {
    auto* h = new symten_tensor;
    h->t = std::move(p);
    return h;
}

hipStream_t S(void* s) { return (hipStream_t)s; }

// ---- plan cache ----------------------------------------------------------
struct PlanCache {
    std::mutex mu;
    std::list<std::pair<std::string, std::shared_ptr<ContractPlan>>> lru;
    std::unordered_map<std::string, decltype(lru)::iterator> map;
    size_t cap = 512;
};
PlanCache& cache() {
    static PlanCache* c = new PlanCache();
    return *c;
}

std::shared_ptr<ContractPlan> get_plan(const Tensor& A, const Tensor& B, int ncon, const int* la, const int* lb,
                                       const int* perm, int prec) {
    std::string key = tensor_signature(A) + "#" + tensor_signature(B) + "#" + std::to_string(ncon) + ":";
    for (int i = 0; i < ncon; ++i) key += std::to_string(la[i]) + "," + std::to_string(lb[i]) + ";";
    const int ro = A.rank() + B.rank() - 2 * ncon;
    key += "p";
    if (perm) for (int j = 0; j < ro; ++j) key += std::to_string(perm[j]) + ",";
    key += "#" + std::to_string(prec);
    PlanCache& C = cache();
    {
        std::lock_guard<std::mutex> lk(C.mu);
        auto it = C.map.find(key);
        if (it != C.map.end()) {
            C.lru.splice(C.lru.begin(), C.lru, it->second);
            return it->second->second;
        }
    }
    auto p = plan_contraction(A, B, ncon, la, lb, perm, prec);
    std::lock_guard<std::mutex> lk(C.mu);
    C.lru.emplace_front(key, p);
    C.map[key] = C.lru.begin();
    while (C.lru.size() > C.cap) {
        C.map.erase(C.lru.back().first);
        C.lru.pop_back();
    }
    return p;
}

}  // namespace

std::shared_ptr<ContractPlan> cached_plan(const Tensor& A, const Tensor& B, int ncon, const int* la, const int* lb,
                                          const int* perm, int prec) {
    return get_plan(A, B, ncon, la, lb, perm, prec);
}

namespace {
struct Contracted {
    TensorPtr t;
    std::shared_ptr<ContractPlan> plan;
};

Contracted contract(const Tensor& A, const Tensor& B, std::initializer_list<int> la, std::initializer_list<int> lb,
                    const std::vector<int>& perm, int prec, hipStream_t s) {
    std::vector<int> a(la), b(lb);
    auto p = get_plan(A, B, (int)a.size(), a.data(), b.data(), perm.empty() ? nullptr : perm.data(), prec);
    return {run_contraction(*p, A, B, s), p};
}

void add_info(symten_plan_stats& acc, const symten_plan_stats& x) {
    acc.pairs += x.pairs;
    acc.out_blocks += x.out_blocks;
    acc.useful_flops += x.useful_flops;
    acc.groups += x.groups;
    acc.gemm_flops += x.gemm_flops;
    acc.max_m = std::max(acc.max_m, x.max_m);
    acc.max_n = std::max(acc.max_n, x.max_n);
    acc.max_k = std::max(acc.max_k, x.max_k);
}

// Legs of the three steps of corner `which` (see the header).
struct CornerSpec {
    std::vector<int> l1a, l1b, l2a, l2b, l3a, l3b;
};
CornerSpec corner_spec(int which) {
    switch (which) {
        case 1: return {{1}, {0}, {0}, {2}, {3, 0}, {0, 1}};
        case 2: return {{0}, {2}, {0}, {0}, {1, 2}, {1, 2}};
        case 3: return {{1}, {0}, {0}, {2}, {3, 0}, {2, 3}};
        case 4: return {{0}, {2}, {0}, {0}, {2, 1}, {0, 3}};
        default: fail(SYMTEN_E_INVAL, "enlarged corner: which must be 1..4");
    }
}

struct CornerResult {
    TensorPtr step1, step2, corner;
    symten_plan_stats info{};
};

CornerResult corner(int which, const Tensor& C, const Tensor& Ta, const Tensor& Tb, const Tensor& a, int prec,
                    hipStream_t s) {
    CornerSpec sp = corner_spec(which);
    CornerResult r;
    auto run = [&](const Tensor& X, const Tensor& Y, const std::vector<int>& la, const std::vector<int>& lb) {
        auto p = get_plan(X, Y, (int)la.size(), la.data(), lb.data(), nullptr, prec);
        add_info(r.info, p->info);
        return run_contraction(*p, X, Y, s);
    };
    r.step1 = run(C, Ta, sp.l1a, sp.l1b);
    r.step2 = run(*r.step1, Tb, sp.l2a, sp.l2b);
    r.corner = run(*r.step2, a, sp.l3a, sp.l3b);
    return r;
}

// The same corner with the site tensor absorbed as two layers (the paper's
// single-layer alternative, Sec. 3.2): the two D^2 legs of step 2 that meet a
// are split into (ket, bra) legs, A takes the ket legs, A* (A with every leg
// direction reversed, same data: A is real) the bra legs and the physical leg,
// and the two free (ket, bra) pairs are fused back into the double-layer legs
// of a.  Same legs, order and values as corner().
// The planned steps of one single-layer corner, reused while the inputs'
// layouts repeat (as in a CTM run): no host planning or synchronisation on
// later calls.
struct SingleLayerPipe {
    std::shared_ptr<ContractPlan> p[4];        // C.Ta, .Tb, .A (ket), .A* (bra, phys)
    std::shared_ptr<GatherPlan> split[2], fuse[2];
    symten_plan_stats info{};
};
std::mutex g_sl_mu;
std::map<std::string, std::shared_ptr<SingleLayerPipe>> g_sl_cache;

CornerResult corner_single_layer(int which, const Tensor& C, const Tensor& Ta, const Tensor& Tb, const Tensor& A,
                                 int prec, hipStream_t s) {
    if (A.rank() != 5 || !abelian(A.group)) fail(SYMTEN_E_INVAL, "single-layer corner: A is a rank-5 abelian tensor");
    for (const Tensor* t : {&C, &Ta, &Tb, &A}) check_device_tensor(*t, "single-layer corner");
    const int cm = charge_mod(A.group);
    // A* = A with every leg direction reversed: the bra leg of a bond carries
    // the ket's labels, so the data and labels stay and the flux changes sign
    auto As = std::make_shared<Tensor>(A);
    for (auto& L : As->legs) L.dir = -L.dir;
    As->flux = cnorm(-A.flux, cm);
    const std::string key = std::to_string(which) + "#" + std::to_string(prec) + "#" + tensor_signature(C) + "#" +
                            tensor_signature(Ta) + "#" + tensor_signature(Tb) + "#" + tensor_signature(A);
    std::shared_ptr<SingleLayerPipe> pipe;
    {
        std::lock_guard<std::mutex> lk(g_sl_mu);
        auto it = g_sl_cache.find(key);
        if (it != g_sl_cache.end()) pipe = it->second;
    }
    CornerResult r;
    if (pipe) {
        r.step1 = run_contraction(*pipe->p[0], C, Ta, s);
        r.step2 = run_contraction(*pipe->p[1], *r.step1, Tb, s);
        TensorPtr X1 = run_gather_plan(*pipe->split[1], *run_gather_plan(*pipe->split[0], *r.step2, s), s);
        TensorPtr Y = run_contraction(*pipe->p[2], *X1, A, s);
        TensorPtr Z = run_contraction(*pipe->p[3], *Y, *As, s);
        r.corner = run_gather_plan(*pipe->fuse[1], *run_gather_plan(*pipe->fuse[0], *Z, s), s);
        r.info = pipe->info;
        return r;
    }
    pipe = std::make_shared<SingleLayerPipe>();
    CornerSpec sp = corner_spec(which);
    int np = 0;
    auto run = [&](const Tensor& X, const Tensor& Y, const std::vector<int>& la, const std::vector<int>& lb) {
        auto p = get_plan(X, Y, (int)la.size(), la.data(), lb.data(), nullptr, prec);
        add_info(r.info, p->info);
        pipe->p[np++] = p;
        return run_contraction(*p, X, Y, s);
    };
    r.step1 = run(C, Ta, sp.l1a, sp.l1b);
    r.step2 = run(*r.step1, Tb, sp.l2a, sp.l2b);
    // split the two legs that meet a, the later one first
    const int nX = r.step2->rank();
    const std::vector<int> xs = sp.l3a, as = sp.l3b;   // X leg xs[i] meets a leg as[i]
    const int first = xs[0] > xs[1] ? 0 : 1;
    TensorPtr X1 = r.step2;
    int ns = 0;
    for (int i : {first, 1 - first}) {
        pipe->split[ns] = plan_unfuse(*X1, xs[i], A.legs[as[i] + 1]);
        X1 = run_gather_plan(*pipe->split[ns++], *X1, s);
    }
    // ket position of absorbed leg i in X1: one further per split leg before it
    auto ket_pos = [&](int i) { return xs[i] + (xs[1 - i] < xs[i] ? 1 : 0); };
    const std::vector<int> kx = {ket_pos(0), ket_pos(1)};
    // Y = X1 . A over the ket legs: [X1's other legs, phys, A's free virtual legs]
    TensorPtr Y = run(*X1, A, kx, {as[0] + 1, as[1] + 1});
    std::vector<int> x1free;
    for (int l = 0; l < X1->rank(); ++l)
        if (l != kx[0] && l != kx[1]) x1free.push_back(l);
    auto ypos = [&](int x1leg) { return (int)(std::find(x1free.begin(), x1free.end(), x1leg) - x1free.begin()); };
    const int ysig = (int)x1free.size();
    // Z = Y . A* over the bra legs and the physical leg:
    // [X's other legs, ket_0, ket_1, bra_0, bra_1] for a's free legs 0, 1
    TensorPtr Z = run(*Y, *As, {ypos(kx[0] + 1), ypos(kx[1] + 1), ysig}, {as[0] + 1, as[1] + 1, 0});
    std::vector<int> afree;
    for (int l = 0; l < 4; ++l)
        if (l != as[0] && l != as[1]) afree.push_back(l);
    const int nXf = nX - 2;
    TensorPtr out = Z;
    for (int i = 0; i < 2; ++i) {
        std::vector<int> ket, bra;
        Leg F;
        double_layer_states(A.legs[afree[i] + 1], ket, bra, F, cm);
        F.dir = A.legs[afree[i] + 1].dir;
        // after i fusions: [X's other legs, F_0 .. F_(i-1), ket_i .. ket_1, bra_i .. bra_1]
        pipe->fuse[i] = plan_refuse(*out, nXf + i, nXf + 2, F);
        out = run_gather_plan(*pipe->fuse[i], *out, s);
    }
    r.corner = out;
    pipe->info = r.info;
    std::lock_guard<std::mutex> lk(g_sl_mu);
    if (g_sl_cache.size() > 64) g_sl_cache.clear();   // plans keep their own references
    g_sl_cache[key] = pipe;
    return r;
}

// Several independent contractions in one gather + one grouped-GEMM launch.
struct ContractSpec {
    const Tensor* A;
    const Tensor* B;
    std::vector<int> la, lb, perm;
};
std::vector<Contracted> contract_batched(const std::vector<ContractSpec>& specs, int prec, hipStream_t s) {
    std::vector<std::shared_ptr<ContractPlan>> plans;
    std::vector<const Tensor*> As, Bs;
    for (auto& c : specs) {
        plans.push_back(get_plan(*c.A, *c.B, (int)c.la.size(), c.la.data(), c.lb.data(),
                                 c.perm.empty() ? nullptr : c.perm.data(), prec));
        As.push_back(c.A);
        Bs.push_back(c.B);
    }
    std::vector<TensorPtr> outs = run_contractions_batched(plans, As, Bs, s);
    std::vector<Contracted> r;
    for (size_t i = 0; i < specs.size(); ++i) r.push_back({outs[i], plans[i]});
    return r;
}

// Corners `which` (inputs C, Ta, Tb each), step by step across all of them.
std::vector<CornerResult> corners_batched(const std::vector<int>& which,
                                          const std::vector<std::array<const Tensor*, 3>>& in, const Tensor& a,
                                          int prec, hipStream_t s, const std::vector<const Tensor*>* as = nullptr) {
    const size_t n = which.size();
    std::vector<CornerResult> res(n);
    std::vector<CornerSpec> sp;
    for (int w : which) sp.push_back(corner_spec(w));
    for (int step = 0; step < 3; ++step) {
        std::vector<ContractSpec> cs;
        for (size_t i = 0; i < n; ++i) {
            if (step == 0) cs.push_back({in[i][0], in[i][1], sp[i].l1a, sp[i].l1b, {}});
            else if (step == 1) cs.push_back({res[i].step1.get(), in[i][2], sp[i].l2a, sp[i].l2b, {}});
            else cs.push_back({res[i].step2.get(), as ? (*as)[i] : &a, sp[i].l3a, sp[i].l3b, {}});
        }
        std::vector<Contracted> r = contract_batched(cs, prec, s);
        for (size_t i = 0; i < n; ++i) {
            add_info(res[i].info, r[i].plan->info);
            (step == 0 ? res[i].step1 : step == 1 ? res[i].step2 : res[i].corner) = r[i].t;
        }
    }
    return res;
}

// ---- rocBLAS/rocSOLVER status -------------------------------------------
void rb_check(rocblas_status st, const char* what) {
    if (st != rocblas_status_success)
        fail(SYMTEN_E_LINALG, std::string(what) + " failed: " + rocblas_status_to_string(st));
}

struct Timer {
    hipEvent_t e[8];
    int n = 0;
    bool on = false;
    void init(bool enable) {
        on = enable;
        if (on) for (auto& x : e) HIPCHK(hipEventCreate(&x));
    }
    void mark(hipStream_t s) {
        if (on && n < 8) HIPCHK(hipEventRecord(e[n++], s));
    }
    double ms(int a, int b) {
        float t = 0.f;
        if (!on || b >= n) return 0.0;
        HIPCHK(hipEventElapsedTime(&t, e[a], e[b]));
        return t;
    }
    ~Timer() {
        if (on) for (auto& x : e) (void)hipEventDestroy(x);
    }
};
}  // namespace

}  // namespace symten

using namespace symten;

struct ctm_env {
    TensorPtr C[4], T[4];
    std::vector<double> svals;
    // unit cell of Lx x Ly sites (0: the 1x1 environment above); site (x, y)
    // holds cC[4 (x Ly + y) + i] = C_(i+1) and cT likewise
    int Lx = 0, Ly = 0;
    std::vector<TensorPtr> cC, cT;
    symten_tensor P, Pt;
    rocblas_handle rb = nullptr;
    // side streams for the size classes of the projector eigensolves, which
    // are latency-bound and overlap well (default priority, non-blocking)
    static constexpr int kAux = 3;
    hipStream_t aux[kAux] = {};
    rocblas_handle rb_aux[kAux] = {};
    hipEvent_t ev_start = nullptr, ev_done[kAux] = {};
    // relative spread within which singular values count as one degenerate
    // set at the cut, about ten times the per-value error of the move's
    // precision (set by every move)
    double degen_tol = 1e-8;
    // pinned host staging of the projector stage's one read-back
    char* pinned = nullptr;
    size_t pinned_bytes = 0;
    char* pinned_buffer(size_t bytes) {
        if (bytes > pinned_bytes) {
            if (pinned) HIPCHK(hipHostFree(pinned));
            pinned = nullptr;
            pinned_bytes = 0;
            HIPCHK(hipHostMalloc((void**)&pinned, bytes, hipHostMallocDefault));
            pinned_bytes = bytes;
        }
        return pinned;
    }
    static double degenerate_tol(int prec) {
        switch (prec) {
            case SYMTEN_PREC_F64: return 1e-8;
            case SYMTEN_PREC_F32:
            case SYMTEN_PREC_BF16X6: return 1e-5;
            default: return 1e-4;   // bf16x3, bf16
        }
    }
    ~ctm_env() {
        if (rb) rocblas_destroy_handle(rb);
        for (int i = 0; i < kAux; ++i) {
            if (rb_aux[i]) rocblas_destroy_handle(rb_aux[i]);
            if (ev_done[i]) (void)hipEventDestroy(ev_done[i]);
            if (aux[i]) (void)hipStreamDestroy(aux[i]);
        }
        if (ev_start) (void)hipEventDestroy(ev_start);
        if (pinned) (void)hipHostFree(pinned);
    }
};

// ============================================================ kernels used
// by the projector stage (small, FP64)
namespace symten {
// X[:, j] *= s[j]^e  (col-major, ld)
__global__ void scale_cols_kernel(double* __restrict__ X, int ld, int rows, int cols, const double* __restrict__ s,
                                  double e) {
    const int64_t tot = (int64_t)rows * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int row = (int)(i % rows), col = (int)(i / rows);
        X[row + (int64_t)col * ld] *= pow(s[col], e);
    }
}
// X[i, :] *= s[i]^e
__global__ void scale_rows_kernel(double* __restrict__ X, int ld, int rows, int cols, const double* __restrict__ s,
                                  double e) {
    const int64_t tot = (int64_t)rows * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int row = (int)(i % rows), col = (int)(i / rows);
        X[row + (int64_t)col * ld] *= pow(s[row], e);
    }
}
// Largest mn eigenpairs (syevd returns ascending order, NE of them) as
// singular triplets in descending order.  Jordan-Wielandt: s = lambda,
// u = sqrt2 z[0:ru], v = sqrt2 z[voff:voff+rd]; Gram: s = sqrt(lambda), u = z.
__global__ void eig_to_svd_kernel(const double* __restrict__ Z, int NE, const double* __restrict__ w, int voff,
                                  int mn, int ru, int rd, int jw, double* __restrict__ S, double* __restrict__ U,
                                  double* __restrict__ V) {
    const int j = blockIdx.x;
    if (j >= mn) return;
    const int idx = NE - 1 - j;
    const double lam = fmax(w[idx], 0.0);
    if (threadIdx.x == 0) S[j] = jw ? lam : sqrt(lam);
    const double f = jw ? sqrt(2.0) : 1.0;
    for (int r = threadIdx.x; r < ru; r += blockDim.x) U[r + (int64_t)j * ru] = f * Z[r + (int64_t)idx * NE];
    if (jw)
        for (int r = threadIdx.x; r < rd; r += blockDim.x)
            V[r + (int64_t)j * rd] = f * Z[voff + r + (int64_t)idx * NE];
}
// Singular values of a sector from the eigenvalues w (ascending, NE of
// them) of its Jordan-Wielandt (s = lambda) or Gram (s = sqrt(lambda))
// matrix: the mn largest, descending, negatives (rounding) clamped to 0.
__global__ void eigval_to_s_kernel(const double* __restrict__ w, int NE, int mn, int jw, double* __restrict__ S) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < mn; j += gridDim.x * blockDim.x) {
        const double lam = fmax(w[NE - 1 - j], 0.0);
        S[j] = jw ? lam : sqrt(lam);
    }
}
// Left (and, Jordan-Wielandt, right) singular vectors of the k largest values
// from eigenvectors Zk (NE x k, column j for the j-th largest):
// Jordan-Wielandt u = sqrt2 z[0:ru], v = sqrt2 z[ru:ru+rd]; Gram u = z.
__global__ void vec_to_uv_kernel(const double* __restrict__ Zk, int NE, int k, int ru, int rd, int jw,
                                 double* __restrict__ U, double* __restrict__ V) {
    const int j = blockIdx.x;
    if (j >= k) return;
    const double f = jw ? sqrt(2.0) : 1.0;
    for (int r = threadIdx.x; r < ru; r += blockDim.x) U[r + (int64_t)j * ru] = f * Zk[r + (int64_t)j * NE];
    if (jw)
        for (int r = threadIdx.x; r < rd; r += blockDim.x) V[r + (int64_t)j * rd] = f * Zk[ru + r + (int64_t)j * NE];
}
// Compact Jordan-Wielandt matrix [[0, Y], [Y^T, 0]] of order ru + rd from
// Y (ru x rd, column-major, ld ru).
__global__ void jw_build_compact_kernel(const double* __restrict__ Y, int ru, int rd, double* __restrict__ J) {
    const int N = ru + rd;
    const int64_t tot = (int64_t)N * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i % N), c = (int)(i / N);
        double v = 0.0;
        if (r < ru && c >= ru) v = Y[r + (int64_t)(c - ru) * ru];
        else if (r >= ru && c < ru) v = Y[c + (int64_t)(r - ru) * ru];
        J[i] = v;
    }
}
// Non-finite entries of X (NaN, Inf) are replaced by 0 and reported in
// *flag, so that the eigensolver only ever sees finite matrices; the move
// then fails after the read-back (SYMTEN_E_LINALG).
__global__ void nonfinite_guard_kernel(double* __restrict__ X, int64_t n, int* __restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = X[i];
        if (!isfinite(v)) {
            X[i] = 0.0;
            *flag = 1;
        }
    }
}
// Zero-padded FP64 copies of col-major blocks: dst[j] is N x N.
__global__ void pad_blocks_kernel(PadArgs a, double* __restrict__ dst) {
    const int j = blockIdx.y;
    const int64_t N2 = (int64_t)a.N * a.N;
    const int rows = a.rows[j], cols = a.cols[j];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N2; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i % a.N), c = (int)(i / a.N);
        double v = 0.0;
        if (r < rows && c < cols)
            v = a.src_f64 ? ((const double*)a.src[j])[r + (int64_t)c * rows]
                          : (double)((const float*)a.src[j])[r + (int64_t)c * rows];
        dst[j * N2 + i] = v;
    }
}
__global__ void jw_build_batched_kernel(const double* __restrict__ M, int N, double* __restrict__ J) {
    const int j = blockIdx.y;
    const int N2x = 2 * N;
    const int64_t tot = (int64_t)N2x * N2x;
    const double* Mj = M + (int64_t)j * N * N;
    double* Jj = J + (int64_t)j * tot;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i % N2x), c = (int)(i / N2x);
        double v = 0.0;
        if (r < N && c >= N) v = Mj[r + (int64_t)(c - N) * N];
        else if (r >= N && c < N) v = Mj[c + (int64_t)(r - N) * N];
        Jj[i] = v;
    }
}
static int g1d(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }
void launch_nonfinite_guard(double* X, int64_t n, int* flag, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(nonfinite_guard_kernel, dim3(g1d(n)), dim3(256), 0, st, X, n, flag);
    HIPCHK(hipGetLastError());
}
void launch_scale_cols(double* X, int ld, int rows, int cols, const double* sv, double e, hipStream_t st) {
    if ((int64_t)rows * cols == 0) return;
    hipLaunchKernelGGL(scale_cols_kernel, dim3(g1d((int64_t)rows * cols)), dim3(256), 0, st, X, ld, rows, cols, sv, e);
    HIPCHK(hipGetLastError());
}
void launch_scale_rows(double* X, int ld, int rows, int cols, const double* sv, double e, hipStream_t st) {
    if ((int64_t)rows * cols == 0) return;
    hipLaunchKernelGGL(scale_rows_kernel, dim3(g1d((int64_t)rows * cols)), dim3(256), 0, st, X, ld, rows, cols, sv, e);
    HIPCHK(hipGetLastError());
}
void launch_eig_to_svd(const double* Z, int NE, const double* w, int voff, int mn, int ru, int rd, bool jw,
                       double* S, double* U, double* V, hipStream_t st) {
    if (mn <= 0) return;
    hipLaunchKernelGGL(eig_to_svd_kernel, dim3(mn), dim3(256), 0, st, Z, NE, w, voff, mn, ru, rd, jw ? 1 : 0, S, U,
                       V);
    HIPCHK(hipGetLastError());
}
void launch_eigval_to_s(const double* w, int NE, int mn, bool jw, double* S, hipStream_t st) {
    if (mn <= 0) return;
    hipLaunchKernelGGL(eigval_to_s_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, st, w, NE, mn,
                       jw ? 1 : 0, S);
    HIPCHK(hipGetLastError());
}
void launch_vec_to_uv(const double* Zk, int NE, int k, int ru, int rd, bool jw, double* U, double* V, hipStream_t st) {
    if (k <= 0) return;
    hipLaunchKernelGGL(vec_to_uv_kernel, dim3((unsigned)k), dim3(256), 0, st, Zk, NE, k, ru, rd, jw ? 1 : 0, U, V);
    HIPCHK(hipGetLastError());
}
void launch_jw_build_compact(const double* Y, int ru, int rd, double* J, hipStream_t st) {
    const int64_t N = (int64_t)ru + rd;
    if (N <= 0) return;
    hipLaunchKernelGGL(jw_build_compact_kernel, dim3((unsigned)g1d(N * N)), dim3(256), 0, st, Y, ru, rd, J);
    HIPCHK(hipGetLastError());
}
void launch_pad_blocks(const PadArgs& a, double* dst, hipStream_t st) {
    if (a.count <= 0 || a.N <= 0) return;
    dim3 grid((unsigned)g1d((int64_t)a.N * a.N), (unsigned)a.count);
    hipLaunchKernelGGL(pad_blocks_kernel, grid, dim3(256), 0, st, a, dst);
    HIPCHK(hipGetLastError());
}
void launch_jw_build_batched(const double* M, int N, int count, double* J, hipStream_t st) {
    if (count <= 0 || N <= 0) return;
    dim3 grid((unsigned)g1d(4 * (int64_t)N * N), (unsigned)count);
    hipLaunchKernelGGL(jw_build_batched_kernel, grid, dim3(256), 0, st, M, N, J);
    HIPCHK(hipGetLastError());
}
}  // namespace symten

namespace {

TensorPtr make_desc_tensor(const symten_desc* d) {
    if (!d) fail(SYMTEN_E_INVAL, "null descriptor");
    if (d->group != SYMTEN_U1 && d->group != SYMTEN_SU2 && d->group != SYMTEN_Z2)
        fail(SYMTEN_E_INVAL, "unknown symmetry group");
    if (d->group == SYMTEN_Z2 && d->flux != 0 && d->flux != 1) fail(SYMTEN_E_SYM, "Z2 flux is a parity, 0 or 1");
    if (d->group == SYMTEN_SU2 && d->flux != 0) fail(SYMTEN_E_SYM, "SU(2) tensors are invariant: flux must be 0");
    if (d->rank < 1 || d->rank > SYMTEN_MAX_RANK) fail(SYMTEN_E_INVAL, "rank must be 1..8");
    if (!d->dirs || !d->nsec || !d->labels || !d->dims) fail(SYMTEN_E_INVAL, "null array in descriptor");
    if (d->dtype != SYMTEN_F64 && d->dtype != SYMTEN_F32) fail(SYMTEN_E_INVAL, "dtype must be F64 or F32");
    auto t = std::make_shared<Tensor>();
    t->group = d->group;
    t->flux = d->flux;
    t->dtype = d->dtype;
    int pos = 0;
    for (int l = 0; l < d->rank; ++l) {
        if (d->dirs[l] != 1 && d->dirs[l] != -1) fail(SYMTEN_E_INVAL, "leg direction must be +1 or -1");
        if (d->nsec[l] < 0 || d->nsec[l] > 4096) fail(SYMTEN_E_INVAL, "bad sector count");
        std::vector<std::pair<int, int>> secs;
        for (int s = 0; s < d->nsec[l]; ++s, ++pos) {
            if (d->dims[pos] < 0) fail(SYMTEN_E_INVAL, "negative sector dimension");
            if (d->group == SYMTEN_SU2 && (d->labels[pos] < 0 || d->labels[pos] > 64))
                fail(SYMTEN_E_INVAL, "SU(2) labels are doubled spins 0..64");
            if (d->group == SYMTEN_Z2 && d->labels[pos] != 0 && d->labels[pos] != 1)
                fail(SYMTEN_E_INVAL, "Z2 labels are parities 0, 1");
            if (d->dims[pos] > 0) secs.push_back({d->labels[pos], d->dims[pos]});
        }
        std::sort(secs.begin(), secs.end());
        for (size_t i = 1; i < secs.size(); ++i)
            if (secs[i].first == secs[i - 1].first) fail(SYMTEN_E_INVAL, "duplicate sector label on a leg");
        Leg L;
        L.dir = d->dirs[l];
        for (auto& s : secs) { L.q.push_back(s.first); L.d.push_back(s.second); }
        t->legs.push_back(L);
    }
    t->elems = t->group == SYMTEN_SU2 ? enumerate_blocks_su2(*t) : enumerate_blocks(*t);
    return t;
}

}  // namespace

namespace symten {
namespace {
// One diagonal block of the fused left cut: a U(1) charge or an SU(2) spin.
struct CutSector {
    int key = 0;                 // fused charge Q, or doubled spin 2J
    int weight = 1;              // states per kept value: 1 (U(1)) or 2J+1 (SU(2))
    int n = 0, mu = 0, md = 0;   // rows (left cut) x columns (right cut) of H_u, H_d
    const void* hu = nullptr;    // row-major n x mu and n x md blocks of the halves
    const void* hd = nullptr;    // (storage type of the move)
    // filled by cut_projectors
    int mn = 0;                  // singular values reported (min(n, m))
    int k = 0;                   // kept
    int64_t pbase = 0;           // offset of P[key] (n x k) and P~[key] (k x n)
};
struct ProjOut {
    std::vector<double> sv;      // reduced singular values, sector by sector, descending
    BufferPtr P, Pt;             // FP64, column-major per sector at CutSector::pbase
    int64_t ptot = 0;
    double tot2 = 0, disc2 = 0, smax = 0, gap = 0;
    double cutoff = 0;           // relative truncation floor used (s <= cutoff s_max dropped)
    int64_t flops = 0;
};

// Projectors of the left cut from the blocks of the two halves (FP64).
//
// The scheme factorizes H_u^T = Q_u R_u and H_d^T = Q_d R_d and takes the
// SVD of M = R_u R_d^T.  Since Y = H_u^T H_d = Q_u M Q_d^T, Y has the same
// non-zero singular values, with U_Y = Q_u U and V_Y = Q_d V, so
//   P  = R_d^T V S^-1/2 = H_d V_Y S^-1/2,
//   P~ = S^-1/2 U^T R_u = S^-1/2 U_Y^T H_u^T,
// and no QR factorization is needed: per sector one FP64 GEMM forms Y and
// one symmetric eigensolve gives its singular triplets.  rocSOLVER's
// eigensolver is latency-bound (one launch sequence per column), so the
// sectors are grouped into size classes and each class is solved in one
// strided-batched call: a block (col-major m x n = H^T) is zero-padded to the
// class size N, which leaves Y = diag(Y_A, 0) exact; the padding adds only
// zero singular values.  The classes go round robin over the caller's stream
// and the side streams.  FP64 moves use the Jordan-Wielandt matrix
// [[0, Y], [Y^T, 0]] (eigenpairs +-s, [u; +-v]/sqrt2, no squaring of the
// condition number); the other precisions use Y Y^T (eigenvalues s^2), whose
// extra rounding is far below their own error budget.
//
// Truncation (global over sectors): values in descending order (ties: key
// ascending, then index), each kept while the kept states, counted with the
// sector's weight, stay within chi, stopping at the first that does not fit
// (a multiplet is never split) and at values <= cutoff s_max (1e-14 on the
// FP64 route, sqrt(N eps) on the Gram route).  P~ rows get
// the sign gauge (largest-magnitude entry positive).  One host
// synchronisation (the singular values).

// Work buffers of one cut's eigensolves, enqueued but not yet read back.
struct ProjWork {
    int ru = 0, rd = 0, ld = 0;  // ld: of H_u^T, H_d^T
    int ldy = 0;                 // of Y
    double *HuT = nullptr, *HdT = nullptr, *Y = nullptr;
    int* info = nullptr;         // rocSOLVER's status (vendor route only)
    int* nonfinite = nullptr;    // set when Y held NaN or Inf (zeroed before the solve)
    int prob = -1;               // own route: the sector's problem in the cut set's EighWork
    int ne = 0;                  // own route: order of its eigenproblem
    double* w = nullptr;         // own route: its eigenvalues, ascending
    double* sdev = nullptr;      // own route: its singular values (in the cut's read-back area)
    BufferPtr U, V, S;
    const double* s_ptr() const { return sdev ? sdev : (const double*)S->ptr; }
};
struct ProjPending {
    std::vector<ProjWork> w;
    std::vector<BufferPtr> keep_alive;
    bool aux_used[ctm_env::kAux] = {};
    std::shared_ptr<EighWork> eig;   // own route: shared by the cuts solved together
    // own route: the cut's read-back area, one copy to the host: ints
    // [nonfinite flag, solver status per sector], then doubles from
    // rb_head: per sector its eigenvalues (w_off) and singular values (s_off)
    BufferPtr rb;
    size_t rb_doubles = 0, rb_head = 0;
    std::vector<size_t> w_off, s_off;
};

// One size class of a cut: its blocks zero-padded to N, Y = H_u^T H_d, the
// Jordan-Wielandt (FP64) or Gram matrix, one strided-batched eigensolve and
// the singular triplets, all on stream cs with handle rh.
void solve_class(const std::vector<CutSector>& secs, std::vector<ProjWork>& w, const std::vector<int>& cls, int N,
                 bool f64, hipStream_t cs, rocblas_handle rh, std::vector<BufferPtr>& keep) {
    const double one = 1.0, zero = 0.0;
    const int B = (int)cls.size();
    const size_t N2 = (size_t)N * N;
    // H^T blocks (u, d interleaved) -> padded FP64 matrices
    BufferPtr Hb = device_alloc(8 * N2 * 2 * B);
    PadArgs pa{};
    pa.count = 2 * B;
    pa.N = N;
    pa.src_f64 = f64;
    for (int i = 0; i < B; ++i) {
        const CutSector& b = secs[cls[i]];
        for (int side = 0; side < 2; ++side) {
            pa.src[2 * i + side] = side == 0 ? b.hu : b.hd;
            pa.rows[2 * i + side] = side == 0 ? b.mu : b.md;   // col-major m x n (ld m)
            pa.cols[2 * i + side] = b.n;
        }
    }
    launch_pad_blocks(pa, (double*)Hb->ptr, cs);
    // Y = H_u^T H_d for every block of the class
    BufferPtr Mb = device_alloc(8 * N2 * B);
    rb_check(rocblas_dgemm_strided_batched(rh, rocblas_operation_none, rocblas_operation_transpose, N, N, N,
                                           &one, (const double*)Hb->ptr, N, 2 * N2,
                                           (const double*)Hb->ptr + N2, N, 2 * N2, &zero, (double*)Mb->ptr, N,
                                           N2, B),
             "rocblas_dgemm_strided_batched(Y)");
    const int NE = f64 ? 2 * N : N;
    const size_t NE2 = (size_t)NE * NE;
    BufferPtr Zb = device_alloc(8 * NE2 * B);
    BufferPtr wb = device_alloc(8 * (size_t)NE * B);
    BufferPtr Eb = device_alloc(8 * (size_t)NE * B);
    BufferPtr ib = device_alloc(8 * (size_t)B);
    BufferPtr fb = device_alloc(4);
    launch_fill_zero(fb->ptr, 4, cs);
    launch_nonfinite_guard((double*)Mb->ptr, (int64_t)N2 * B, (int*)fb->ptr, cs);
    if (f64)
        launch_jw_build_batched((const double*)Mb->ptr, N, B, (double*)Zb->ptr, cs);
    else
        rb_check(rocblas_dgemm_strided_batched(rh, rocblas_operation_none, rocblas_operation_transpose, N, N,
                                               N, &one, (const double*)Mb->ptr, N, N2,
                                               (const double*)Mb->ptr, N, N2, &zero, (double*)Zb->ptr, N, N2,
                                               B),
                 "rocblas_dgemm_strided_batched(YY^T)");
    rb_check(rocsolver_dsyevd_strided_batched(rh, rocblas_evect_original, rocblas_fill_upper, NE,
                                              (double*)Zb->ptr, NE, NE2, (double*)wb->ptr, NE,
                                              (double*)Eb->ptr, NE, (rocblas_int*)ib->ptr, B),
             "rocsolver_dsyevd_strided_batched");
    for (int i = 0; i < B; ++i) {
        const CutSector& b = secs[cls[i]];
        ProjWork& x = w[cls[i]];
        x.HuT = (double*)Hb->ptr + 2 * i * N2;          // H_u^T, col-major m x n
        x.HdT = (double*)Hb->ptr + (2 * i + 1) * N2;    // H_d^T
        x.Y = (double*)Mb->ptr + i * N2;
        x.ld = N;
        x.ldy = N;
        x.info = (int*)ib->ptr + i;
        x.nonfinite = (int*)fb->ptr;
        x.S = device_alloc(8 * std::max(1, b.mn));
        x.U = device_alloc(8 * std::max<size_t>(1, (size_t)x.ru * b.mn));
        x.V = device_alloc(8 * std::max<size_t>(1, (size_t)x.rd * b.mn));
        launch_eig_to_svd((const double*)Zb->ptr + i * NE2, NE, (const double*)wb->ptr + (size_t)i * NE, N,
                          b.mn, x.ru, x.rd, f64, (double*)x.S->ptr, (double*)x.U->ptr, (double*)x.V->ptr, cs);
    }
    for (auto& x : {Hb, Mb, Zb, wb, Eb, ib, fb}) keep.push_back(x);
}

// The library's own eigensolver (every eigenproblem of the given cuts fits
// its LDS): per sector, H_u^T and H_d^T as FP64 col-major blocks, Y = H_u^T
// H_d (ru x rd, compact), its Gram or compact Jordan-Wielandt matrix; then
// one set of launches tridiagonalises every matrix of every cut and finds
// all eigenvalues, and each sector's singular values are taken from them.
// Everything is enqueued on s; no host thread, no side stream.
std::vector<ProjPending> issue_solves_own(ctm_env* env, const std::vector<std::vector<CutSector>*>& cuts, bool f64,
                                          hipStream_t s) {
    rb_check(rocblas_set_stream(env->rb, s), "rocblas_set_stream");
    const double one = 1.0, zero = 0.0;
    std::vector<ProjPending> pend(cuts.size());
    std::vector<EighProblem> probs;
    for (size_t c = 0; c < cuts.size(); ++c) {
        std::vector<CutSector>& secs = *cuts[c];
        if (secs.empty()) fail(SYMTEN_E_LINALG, "ctm_move: the halves have no common sector");
        ProjPending& pc = pend[c];
        pc.w.resize(secs.size());
        pc.rb_head = (1 + secs.size() + 1) / 2;   // ints, in doubles
        size_t tot = pc.rb_head;
        for (auto& b : secs) {
            b.mn = std::min(b.n, std::min(b.mu, b.md));
            pc.w_off.push_back(tot);
            tot += f64 ? b.mu + b.md : b.mu;
            pc.s_off.push_back(tot);
            tot += std::max(1, b.mn);
        }
        pc.rb_doubles = tot;
        pc.rb = device_alloc(8 * tot);
        launch_fill_zero(pc.rb->ptr, 8 * (int64_t)pc.rb_head, s);
        pc.keep_alive.push_back(pc.rb);
        int* head = (int*)pc.rb->ptr;
        double* area = (double*)pc.rb->ptr;
        for (size_t i = 0; i < secs.size(); ++i) {
            CutSector& b = secs[i];
            ProjWork& x = pc.w[i];
            x.ru = b.mu;
            x.rd = b.md;
            const int N = std::max(b.n, std::max(b.mu, b.md));
            const size_t N2 = (size_t)N * N;
            BufferPtr Hb = device_alloc(8 * N2 * 2);
            PadArgs pa{};
            pa.count = 2;
            pa.N = N;
            pa.src_f64 = f64;
            pa.src[0] = b.hu;
            pa.rows[0] = b.mu;
            pa.cols[0] = b.n;
            pa.src[1] = b.hd;
            pa.rows[1] = b.md;
            pa.cols[1] = b.n;
            launch_pad_blocks(pa, (double*)Hb->ptr, s);
            x.HuT = (double*)Hb->ptr;
            x.HdT = (double*)Hb->ptr + N2;
            x.ld = N;
            BufferPtr Yb = device_alloc(8 * std::max<size_t>(1, (size_t)b.mu * b.md));
            x.Y = (double*)Yb->ptr;
            x.ldy = std::max(1, b.mu);
            rb_check(rocblas_dgemm(env->rb, rocblas_operation_none, rocblas_operation_transpose, b.mu, b.md, b.n,
                                   &one, x.HuT, N, x.HdT, N, &zero, x.Y, x.ldy),
                     "rocblas_dgemm(Y)");
            x.nonfinite = head;
            launch_nonfinite_guard(x.Y, (int64_t)b.mu * b.md, x.nonfinite, s);
            x.ne = f64 ? b.mu + b.md : b.mu;
            BufferPtr Ab = device_alloc(8 * (size_t)x.ne * x.ne);
            if (f64)
                launch_jw_build_compact(x.Y, b.mu, b.md, (double*)Ab->ptr, s);
            else
                rb_check(rocblas_dgemm(env->rb, rocblas_operation_none, rocblas_operation_transpose, b.mu, b.mu, b.md,
                                       &one, x.Y, x.ldy, x.Y, x.ldy, &zero, (double*)Ab->ptr, x.ne),
                         "rocblas_dgemm(YY^T)");
            x.w = area + pc.w_off[i];
            x.sdev = area + pc.s_off[i];
            x.prob = (int)probs.size();
            EighProblem ep;
            ep.n = x.ne;
            ep.lda = x.ne;
            ep.A = (const double*)Ab->ptr;
            ep.w = x.w;
            ep.status = head + 1 + i;
            probs.push_back(ep);
            for (auto& k : {Hb, Yb, Ab}) pc.keep_alive.push_back(k);
        }
    }
    auto wk = eigh_values(probs, s);
    for (size_t c = 0; c < cuts.size(); ++c) {
        pend[c].eig = wk;
        std::vector<CutSector>& secs = *cuts[c];
        for (size_t i = 0; i < secs.size(); ++i) {
            ProjWork& x = pend[c].w[i];
            launch_eigval_to_s(x.w, x.ne, secs[i].mn, f64, x.sdev, s);
        }
    }
    return pend;
}

bool own_solver_fits(const std::vector<std::vector<CutSector>*>& cuts, bool f64) {
    for (auto* secs : cuts)
        for (auto& b : *secs)
            if (!eigh_fits(f64 ? b.mu + b.md : b.mu)) return false;
    return true;
}

// Enqueues the eigensolves of every sector of the given cuts (no host
// synchronisation).  Each cut's sectors are grouped into size classes
// (largest first); the classes of all cuts go round robin over the caller's
// stream and the side streams, so that the largest classes of several cuts
// land on different streams.  `start` is recorded on s by the caller once the
// halves of every cut are enqueued; side streams wait for it.  Enqueueing
// rocSOLVER's eigensolver is host-bound (about two thirds of its device time
// at n = 696), so every stream's classes are enqueued by a host thread of
// their own, each with the stream's own rocBLAS handle.
std::vector<ProjPending> issue_solves(ctm_env* env, const std::vector<std::vector<CutSector>*>& cuts, bool f64,
                                      hipStream_t s, hipEvent_t start) {
    if (own_solver_fits(cuts, f64)) return issue_solves_own(env, cuts, f64, s);
    rb_check(rocblas_set_stream(env->rb, s), "rocblas_set_stream");
    constexpr int kSlots = ctm_env::kAux + 1;
    struct SolveClass {
        int cut, N, slot;
        std::vector<int> cls;
        std::vector<BufferPtr> keep;
    };
    std::vector<ProjPending> pend(cuts.size());
    std::vector<SolveClass> classes;
    int rr = 0;
    for (size_t c = 0; c < cuts.size(); ++c) {
        std::vector<CutSector>& secs = *cuts[c];
        if (secs.empty()) fail(SYMTEN_E_LINALG, "ctm_move: the halves have no common sector");
        pend[c].w.resize(secs.size());
        std::vector<int> order(secs.size());
        std::iota(order.begin(), order.end(), 0);
        for (size_t i = 0; i < secs.size(); ++i) {
            pend[c].w[i].ru = secs[i].mu;                                // rows of U_Y
            pend[c].w[i].rd = secs[i].md;                                // rows of V_Y
            secs[i].mn = std::min(secs[i].n, std::min(secs[i].mu, secs[i].md));   // rank bound
        }
        auto dim = [&](int i) { return std::max(secs[i].n, std::max(secs[i].mu, secs[i].md)); };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return dim(x) > dim(y); });
        size_t pos = 0;
        while (pos < order.size()) {
            SolveClass k;
            k.cut = (int)c;
            k.N = dim(order[pos]);
            while (pos < order.size() && (int)k.cls.size() < kMaxPadBatch / 2 && 2 * dim(order[pos]) >= k.N)
                k.cls.push_back(order[pos++]);
            k.slot = rr++ % kSlots;
            if (k.slot > 0) pend[c].aux_used[k.slot - 1] = true;
            classes.push_back(std::move(k));
        }
    }
    bool waiting[ctm_env::kAux] = {};
    for (auto& k : classes)
        if (k.slot > 0 && !waiting[k.slot - 1]) {
            HIPCHK(hipStreamWaitEvent(env->aux[k.slot - 1], start, 0));
            waiting[k.slot - 1] = true;
        }
    auto run_slot = [&](int slot) {
        hipStream_t cs = slot == 0 ? s : env->aux[slot - 1];
        StreamScope scope(cs);   // work buffers of this slot are used on cs
        rocblas_handle rh = slot == 0 ? env->rb : env->rb_aux[slot - 1];
        for (auto& k : classes)
            if (k.slot == slot) solve_class(*cuts[k.cut], pend[k.cut].w, k.cls, k.N, f64, cs, rh, k.keep);
    };
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::exception_ptr err[kSlots];
    std::vector<std::thread> workers;
    std::vector<int> inline_slots = {0};
    for (int slot = 1; slot < kSlots; ++slot) {
        if (!waiting[slot - 1]) continue;
        try {
            workers.emplace_back([&, slot] {
                try {
                    HIPCHK(hipSetDevice(dev));
                    run_slot(slot);
                } catch (...) {
                    err[slot] = std::current_exception();
                }
            });
        } catch (const std::system_error&) {
            inline_slots.push_back(slot);   // no thread to spare: enqueue it from this one
        }
    }
    for (int slot : inline_slots) {
        try {
            run_slot(slot);
        } catch (...) {
            err[slot] = std::current_exception();
            break;
        }
    }
    for (auto& t : workers) t.join();
    for (auto& e : err)
        if (e) {
            // solves enqueued by the other threads may still run: drain the
            // streams before their work buffers go back to the pool
            (void)hipStreamSynchronize(s);
            for (int a = 0; a < ctm_env::kAux; ++a)
                if (waiting[a]) (void)hipStreamSynchronize(env->aux[a]);
            (void)hipGetLastError();
            std::rethrow_exception(e);
        }
    for (auto& k : classes)
        for (auto& x : k.keep) pend[k.cut].keep_alive.push_back(x);
    return pend;
}

// Joins the side streams, reads the singular values back (the one host
// synchronisation), truncates and forms P and P~ on s.
ProjOut finish_projectors(ctm_env* env, std::vector<CutSector>& secs, ProjPending& pend, int chi, bool f64,
                          hipStream_t s) {
    rb_check(rocblas_set_stream(env->rb, s), "rocblas_set_stream");
    std::vector<ProjWork>& w = pend.w;
    ProjOut out;
    std::vector<int> sv_off;
    std::vector<std::vector<double>> w_host(secs.size());
    {
        for (int a = 0; a < ctm_env::kAux; ++a)
            if (pend.aux_used[a]) {
                HIPCHK(hipEventRecord(env->ev_done[a], env->aux[a]));
                HIPCHK(hipStreamWaitEvent(s, env->ev_done[a], 0));
            }
        // singular values and status to the host (the one synchronisation)
        int tot = 0;
        for (auto& c : secs) { sv_off.push_back(tot); tot += c.mn; }
        out.sv.resize(tot);
        std::vector<int> infos(secs.size()), bad(secs.size());
        if (pend.eig) {
            // own route: the cut's whole read-back area in one copy
            const size_t bytes = 8 * pend.rb_doubles;
            char* h = env->pinned_buffer(bytes);
            HIPCHK(hipMemcpyAsync(h, pend.rb->ptr, bytes, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            const int* head = (const int*)h;
            const double* area = (const double*)h;
            for (size_t i = 0; i < secs.size(); ++i) {
                bad[i] = head[0];
                if (head[1 + i])
                    fail(SYMTEN_E_HIP, "ctm_move: the workgroups of an eigensolve did not meet at a barrier");
                w_host[i].assign(area + pend.w_off[i], area + pend.w_off[i] + pend.w[i].ne);
                std::copy(area + pend.s_off[i], area + pend.s_off[i] + secs[i].mn, out.sv.begin() + sv_off[i]);
            }
        } else {
            for (size_t i = 0; i < secs.size(); ++i) {
                if (secs[i].mn)
                    HIPCHK(hipMemcpyAsync(out.sv.data() + sv_off[i], pend.w[i].S->ptr, 8 * secs[i].mn,
                                          hipMemcpyDeviceToHost, s));
                if (pend.w[i].info)
                    HIPCHK(hipMemcpyAsync(&infos[i], pend.w[i].info, sizeof(int), hipMemcpyDeviceToHost, s));
                HIPCHK(hipMemcpyAsync(&bad[i], pend.w[i].nonfinite, sizeof(int), hipMemcpyDeviceToHost, s));
            }
            HIPCHK(hipStreamSynchronize(s));
        }
        for (size_t i = 0; i < secs.size(); ++i)
            if (bad[i]) fail(SYMTEN_E_LINALG, "ctm_move: NaN or Inf in the halves of the cut");
        for (size_t i = 0; i < secs.size(); ++i)
            if (pend.w[i].info && infos[i] != 0) fail(SYMTEN_E_LINALG, "rocsolver_dsyevd did not converge");
        for (double v : out.sv)
            if (!std::isfinite(v)) fail(SYMTEN_E_LINALG, "non-finite singular value");
    }
    // ---- truncation ------------------------------------------------------
    struct SV { double s; int key, sec, j; };
    std::vector<SV> all;
    for (size_t i = 0; i < secs.size(); ++i)
        for (int j = 0; j < secs[i].mn; ++j) all.push_back({out.sv[sv_off[i] + j], secs[i].key, (int)i, j});
    std::sort(all.begin(), all.end(), [](const SV& x, const SV& y) {
        if (x.s != y.s) return x.s > y.s;
        if (x.key != y.key) return x.key < y.key;
        return x.j < y.j;
    });
    out.smax = all.empty() ? 0.0 : all[0].s;
    // values at or below the route's noise floor are dropped: the FP64
    // (Jordan-Wielandt) route keeps the reading's 1e-14 s_max; the Gram route
    // takes s = sqrt(eig(Y Y^T)), whose eigenvalues carry an absolute error of
    // about N eps s_max^2 (N the order of the largest solve), so singular
    // values below sqrt(N eps) s_max are not resolved there
    double cutoff = 1e-14;
    if (!f64) {
        int nmax = 1;
        for (auto& c : secs) nmax = std::max(nmax, std::max(c.mu, c.md));
        cutoff = std::sqrt(nmax * 0x1p-52);
    }
    out.cutoff = cutoff;
    int nkeep = 0, states = 0;
    while (nkeep < (int)all.size() && all[nkeep].s > cutoff * out.smax &&
           states + secs[all[nkeep].sec].weight <= chi) {
        states += secs[all[nkeep].sec].weight;
        ++nkeep;
    }
    // a set of (near-)degenerate values is never split at the cut: values
    // within env->degen_tol (relative) of the last kept one are dropped with it
    while (nkeep > 1 && nkeep < (int)all.size() && all[nkeep].s >= (1.0 - env->degen_tol) * all[nkeep - 1].s) {
        states -= secs[all[nkeep - 1].sec].weight;
        --nkeep;
    }
    if (nkeep == 0) fail(SYMTEN_E_LINALG, "ctm_move: no singular value above the cutoff");
    for (size_t i = 0; i < all.size(); ++i) {
        const double v = secs[all[i].sec].weight * all[i].s * all[i].s;
        out.tot2 += v;
        if ((int)i >= nkeep) out.disc2 += v;
    }
    out.gap = nkeep < (int)all.size() ? (all[nkeep - 1].s - all[nkeep].s) / out.smax : INFINITY;
    for (int i = 0; i < nkeep; ++i) secs[all[i].sec].k += 1;
    // the kept set of a sector is a prefix of its descending list
    if (pend.eig) {
        // own route: eigenvectors of the kept values only, then u (and v)
        std::vector<int> kv(eigh_problems(*pend.eig), 0);
        std::vector<double*> zs(kv.size(), nullptr);
        std::vector<const double*> wh(kv.size(), nullptr);
        std::vector<BufferPtr> zb(secs.size());
        for (size_t i = 0; i < secs.size(); ++i) {
            ProjWork& x = w[i];
            const int k = secs[i].k;
            if (k == 0) continue;
            zb[i] = device_alloc(8 * (size_t)x.ne * k);
            kv[x.prob] = k;
            zs[x.prob] = (double*)zb[i]->ptr;
            wh[x.prob] = w_host[i].data();
        }
        eigh_vectors(*pend.eig, kv, zs, wh, s);
        for (size_t i = 0; i < secs.size(); ++i) {
            ProjWork& x = w[i];
            const int k = secs[i].k;
            if (k == 0) continue;
            x.U = device_alloc(8 * (size_t)x.ru * k);
            x.V = device_alloc(8 * (size_t)x.rd * k);
            launch_vec_to_uv((const double*)zb[i]->ptr, x.ne, k, x.ru, x.rd, f64, (double*)x.U->ptr,
                             (double*)x.V->ptr, s);
        }
    }
    // ---- P = H_d V_k S^-1/2 (n x k), P~ = S^-1/2 U_k^T H_u^T (k x n) -------
    for (auto& c : secs) {
        c.pbase = out.ptot;
        out.ptot += (int64_t)c.n * c.k;
    }
    out.P = device_alloc(8 * std::max<int64_t>(out.ptot, 1));
    out.Pt = device_alloc(8 * std::max<int64_t>(out.ptot, 1));
    const double one = 1.0, zero = 0.0;
    for (size_t i = 0; i < secs.size(); ++i) {
        const CutSector& c = secs[i];
        ProjWork& x = w[i];
        out.flops += 2LL * x.ru * x.rd * c.n;
        if (c.k == 0) continue;
        const int n = c.n, k = c.k;
        double* Pq = (double*)out.P->ptr + c.pbase;
        double* Ptq = (double*)out.Pt->ptr + c.pbase;
        if (!f64) {
            // Gram path: V_k = Y^T U_k S_k^-1  (rd x k, ld rd)
            rb_check(rocblas_dgemm(env->rb, rocblas_operation_transpose, rocblas_operation_none, x.rd, k, x.ru, &one,
                                   (const double*)x.Y, x.ldy, (const double*)x.U->ptr, x.ru, &zero, (double*)x.V->ptr,
                                   x.rd),
                     "rocblas_dgemm(V)");
            launch_scale_cols((double*)x.V->ptr, x.rd, x.rd, k, x.s_ptr(), -1.0, s);
        }
        // P = H_d V_k S^-1/2  (n x k, ld n; H_d = (H_d^T)^T)
        rb_check(rocblas_dgemm(env->rb, rocblas_operation_transpose, rocblas_operation_none, n, k, x.rd, &one,
                               (const double*)x.HdT, x.ld, (const double*)x.V->ptr, x.rd, &zero, Pq, n),
                 "rocblas_dgemm(P)");
        launch_scale_cols(Pq, n, n, k, x.s_ptr(), -0.5, s);
        // P~ = S^-1/2 U_k^T H_u^T  (k x n, ld k)
        rb_check(rocblas_dgemm(env->rb, rocblas_operation_transpose, rocblas_operation_none, k, n, x.ru, &one,
                               (const double*)x.U->ptr, x.ru, (const double*)x.HuT, x.ld, &zero, Ptq, k),
                 "rocblas_dgemm(Pt)");
        launch_scale_rows(Ptq, k, k, n, x.s_ptr(), -0.5, s);
        launch_sign_fix_rows(Ptq, k, k, n, Pq, n, s);
    }
    // the work buffers go back to the pool here; later launches that reuse
    // them are ordered after these on the same stream
    return out;
}

ProjOut cut_projectors(ctm_env* env, std::vector<CutSector>& secs, int chi, bool f64, hipStream_t s) {
    HIPCHK(hipEventRecord(env->ev_start, s));
    std::vector<ProjPending> pend = issue_solves(env, {&secs}, f64, s, env->ev_start);
    return finish_projectors(env, secs, pend[0], chi, f64, s);
}

void fill_cut_stats(ctm_move_stats* st, const std::vector<CutSector>& secs, const ProjOut& po) {
    int nk = 0;
    for (auto& c : secs)
        if (c.k > 0 && nk < CTM_MAX_SECTORS) { st->charge[nk] = c.key; st->kept[nk] = c.k; ++nk; }
    st->nsec = nk;
    st->n_sv_sectors = std::min<int>((int)secs.size(), CTM_MAX_SECTORS);
    for (int i = 0; i < st->n_sv_sectors; ++i) { st->sv_charge[i] = secs[i].key; st->sv_count[i] = secs[i].mn; }
    st->trunc_err = po.tot2 > 0 ? po.disc2 / po.tot2 : 0.0;
    st->s_max = po.smax;
    st->cutoff = po.cutoff;
    st->gap = po.gap;
    st->flops_proj = po.flops;
}
}  // namespace
}  // namespace symten

namespace symten {
namespace {
// ---------------------------------------------------------------- SU(2) move
Leg dual_leg(const Leg& l) {
    Leg d = l;
    d.dir = -l.dir;
    return d;
}

// Fusion isometry F[a, b, f] (SU(2)): f's multiplets of spin J are the pairs
// (multiplet of a with spin ja, multiplet of b with spin jb) with J in ja x jb,
// ordered by (ja, jb) then row-major (i_a, i_b).  Reduced block (ja, jb, J) is
// w * delta(f, pair index) with w = sqrt((2J+1)/(2K+1)) for the block's tree
// root K, which makes the dense F unitary (its basis tensors restricted to a
// fixed f state have squared norm (2K+1)/(2J+1) by Schur's lemma).  Cached
// per leg structure.
TensorPtr fusion_isometry(const Leg& la, const Leg& lb, int fdir, int dtype, hipStream_t s) {
    static std::mutex mu;
    static std::map<std::string, TensorPtr> cache;
    std::ostringstream key;
    for (const Leg* l : {&la, &lb}) {
        key << l->dir << ":";
        for (size_t i = 0; i < l->q.size(); ++i) key << l->q[i] << "x" << l->d[i] << ",";
        key << ";";
    }
    key << fdir << "/" << dtype;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key.str());
    if (it != cache.end()) return it->second;
    // fused multiplets and the position of each (ja, jb) pair inside J
    std::map<int, int> nJ;
    std::map<std::array<int, 3>, int> base;
    for (size_t ia = 0; ia < la.q.size(); ++ia)
        for (size_t ib = 0; ib < lb.q.size(); ++ib)
            for (int J = std::abs(la.q[ia] - lb.q[ib]); J <= la.q[ia] + lb.q[ib]; J += 2) {
                base[{la.q[ia], lb.q[ib], J}] = nJ[J];
                nJ[J] += la.d[ia] * lb.d[ib];
            }
    Leg f;
    f.dir = fdir;
    for (auto& kv : nJ) { f.q.push_back(kv.first); f.d.push_back(kv.second); }
    auto F = std::make_shared<Tensor>();
    F->group = SYMTEN_SU2;
    F->flux = 0;
    F->dtype = dtype;
    F->legs = {la, lb, f};
    F->elems = enumerate_blocks_su2(*F);
    std::vector<double> host((size_t)std::max<int64_t>(F->elems, 1), 0.0);
    for (const Block& b : F->blocks) {
        const int ja = b.q[0], jb = b.q[1], J = b.q[2], K = b.tree.back();
        const double w = std::sqrt((J + 1.0) / (K + 1.0));
        const int na = b.shape[0], nb = b.shape[1];
        const int b0 = base.at({ja, jb, J});
        for (int x = 0; x < na; ++x)
            for (int y = 0; y < nb; ++y)
                host[b.offset + x * b.stride[0] + y * b.stride[1] + (int64_t)(b0 + x * nb + y) * b.stride[2]] = w;
    }
    const size_t es = F->esize();
    F->buf = device_alloc(std::max<int64_t>(F->elems, 1) * es);
    F->meta_only = false;
    if (dtype == SYMTEN_F64) {
        HIPCHK(hipMemcpy(F->buf->ptr, host.data(), F->elems * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> h32(host.begin(), host.end());
        HIPCHK(hipMemcpy(F->buf->ptr, h32.data(), F->elems * 4, hipMemcpyHostToDevice));
    }
    (void)s;
    cache[key.str()] = F;
    return F;
}

// The same tensor with every leg reversed.  A real invariant tensor stays
// invariant under the conjugate transformation law, and its basis tensor
// sum_M C_in C_out is symmetric in the two chains, so only the tree labels
// change: (in intermediates, out intermediates, K) -> (out, in, K).  Shares
// the buffer.
TensorPtr flip_all(const TensorPtr& t) {
    auto r = std::make_shared<Tensor>(*t);
    int nin = 0, nout = 0;
    for (auto& l : r->legs) {
        (l.dir > 0 ? nin : nout) += 1;
        l.dir = -l.dir;
    }
    const int mi = std::max(0, nin - 2), mo = std::max(0, nout - 2);
    for (auto& b : r->blocks) {
        std::vector<int> tr(b.tree.begin() + mi, b.tree.begin() + mi + mo);
        tr.insert(tr.end(), b.tree.begin(), b.tree.begin() + mi);
        tr.push_back(b.tree.back());
        b.tree = tr;
    }
    std::sort(r->blocks.begin(), r->blocks.end(),
              [](const Block& x, const Block& y) { return std::tie(x.q, x.tree) < std::tie(y.q, y.tree); });
    r->rebuild_index();
    return r;
}

// X <- X / |X|_F for an SU(2) tensor: the dense norm is
// sum over blocks of (2K+1) |m_b|^2 (basis tensors of different trees are
// orthogonal, |c|^2 = 2K+1).  FP64 two-pass reduction over a weighted copy.
void normalise_su2(Tensor& X, bool f64, hipStream_t s) {
    std::vector<CopyTask> tasks;
    int64_t pos = 0;
    for (const Block& b : X.blocks) {
        if (b.size == 0) continue;
        std::vector<int64_t> ds(b.shape.size());
        int64_t st = 1;
        for (int l = (int)b.shape.size() - 1; l >= 0; --l) { ds[l] = st; st *= b.shape[l]; }
        tasks.push_back(make_copy_task(0, b.offset, 1, pos, b.shape, b.stride, ds, std::sqrt(b.tree.back() + 1.0)));
        pos += b.size;
    }
    if (tasks.empty()) return;
    BufferPtr tmp = device_alloc(pos * X.esize());
    validate_tasks(tasks, {X.elems, pos});
    std::vector<int64_t> prefix;
    copy_prefix(tasks, prefix);
    BufferPtr dt, dp;
    upload_sync(dt, tasks.data(), tasks.size() * sizeof(CopyTask));
    upload_sync(dp, prefix.data(), prefix.size() * sizeof(int64_t));
    copy_launch_arg((const CopyTask*)dt->ptr, (const int64_t*)dp->ptr, (int)tasks.size(), prefix.back(),
                    {X.data(), tmp->ptr}, f64, f64 ? 1 : 0, s);
    BufferPtr red = device_alloc(8 * (1 + 512));
    launch_sumsq(tmp->ptr, f64, pos, (double*)red->ptr, s);
    launch_scale_by_inv_sqrt(X.data(), f64, X.elems, (const double*)red->ptr, s);
    HIPCHK(hipStreamSynchronize(s));   // descriptor and scratch buffers go back to the pool
}

// One left move on SU(2) reduced tensors.  Corners, halves and the
// renormalisation are the U(1) move's contractions (recoupling scalars in
// the gathers).  For the projectors the two legs of each cut are fused by a
// unitary isometry into one multiplet leg, which turns each half into an
// (in, out) rank-2 tensor: block diagonal in the total spin J of the cut, one
// reduced matrix per J whose dense form is that matrix times the identity on
// 2J+1 states (the rank-2 example of Sec. 2).  The projector stage then runs
// per J exactly as per charge, keeps whole multiplets (2J+1 states each)
// within chi, and the projectors are mapped back through the isometry.
void move_su2(ctm_env* env, Tensor& a, int chi, int prec, ctm_move_stats* st, hipStream_t s) {
    const bool f64 = prec == SYMTEN_PREC_F64;
    const int dtype = f64 ? SYMTEN_F64 : SYMTEN_F32;
    Timer tm;
    tm.init(st != nullptr);
    tm.mark(s);
    Tensor &C1 = *env->C[0], &C2 = *env->C[1], &C3 = *env->C[2], &C4 = *env->C[3];
    Tensor &T1 = *env->T[0], &T2 = *env->T[1], &T3 = *env->T[2], &T4 = *env->T[3];
    std::vector<CornerResult> ks =
        corners_batched({1, 2, 3, 4}, {{&C1, &T1, &T4}, {&C2, &T1, &T2}, {&C3, &T3, &T2}, {&C4, &T3, &T4}}, a, prec, s);
    CornerResult &k1 = ks[0], &k2 = ks[1], &k3 = ks[2], &k4 = ks[3];
    tm.mark(s);
    std::vector<Contracted> hh = contract_batched({{k1.corner.get(), k2.corner.get(), {0, 2}, {0, 2}, {}},
                                                   {k4.corner.get(), k3.corner.get(), {0, 3}, {0, 2}, {}}},
                                                  prec, s);
    const Tensor& Hu = *hh[0].t;   // [x4, d, x2, d2]
    const Tensor& Hd = *hh[1].t;   // [x4, u, x2, u3]
    // the rows of the two halves are the two sides of the cut bond: dual legs
    for (int l = 0; l < 2; ++l)
        if (Hu.legs[l].dir != -Hd.legs[l].dir || !Hu.legs[l].same_sectors(Hd.legs[l]))
            fail(SYMTEN_E_SYM, "ctm_move: upper and lower halves disagree on a cut basis");
    // one dense isometry fuses the rows of both halves (F_L for H_u's leg
    // directions, its reversal for H_d's), so that Y = H_u^T H_d is block
    // diagonal in the fused spin; the columns get isometries of their own
    TensorPtr FL = fusion_isometry(dual_leg(Hu.legs[0]), dual_leg(Hu.legs[1]), 1, dtype, s);
    TensorPtr FLbar = flip_all(FL);
    TensorPtr FRu = fusion_isometry(dual_leg(Hu.legs[2]), dual_leg(Hu.legs[3]), -1, dtype, s);
    TensorPtr FRd = fusion_isometry(dual_leg(Hd.legs[2]), dual_leg(Hd.legs[3]), 1, dtype, s);
    std::vector<Contracted> f1 = contract_batched({{&Hu, FL.get(), {0, 1}, {0, 1}, {}},
                                                   {&Hd, FLbar.get(), {0, 1}, {0, 1}, {}}}, prec, s);   // [x2, d2, L]
    std::vector<Contracted> f2 = contract_batched({{f1[0].t.get(), FRu.get(), {0, 1}, {0, 1}, {}},
                                                   {f1[1].t.get(), FRd.get(), {0, 1}, {0, 1}, {}}}, prec, s);   // [L, R]
    const Tensor& Gu = *f2[0].t;
    const Tensor& Gd = *f2[1].t;
    tm.mark(s);
    // ---- projectors per total spin J of the cut --------------------------
    const size_t es = f64 ? 8 : 4;
    std::vector<CutSector> secs;
    for (const Block& bu : Gu.blocks) {
        const Block* bd = nullptr;
        for (const Block& x : Gd.blocks)
            if (x.q == bu.q && x.tree == bu.tree) bd = &x;
        if (!bd) continue;
        if (bd->shape != bu.shape) fail(SYMTEN_E_SYM, "ctm_move: fused halves disagree on a cut basis");
        for (const Block* x : {&bu, bd})
            if (x->stride[0] != x->shape[1] || x->stride[1] != 1)
                fail(SYMTEN_E_INVAL, "internal: fused half block is not row-major");
        CutSector c;
        c.key = bu.q[0];
        c.weight = bu.q[0] + 1;
        c.n = bu.shape[0];
        c.mu = c.md = bu.shape[1];
        c.hu = (const char*)Gu.data() + bu.offset * es;
        c.hd = (const char*)Gd.data() + bd->offset * es;
        secs.push_back(c);
    }
    ProjOut po = cut_projectors(env, secs, chi, f64, s);
    // P''[L out, k in] (n x k col-major per J), P~''[k out, L in] (k x n)
    auto P2 = std::make_shared<Tensor>();
    auto Pt2 = std::make_shared<Tensor>();
    Leg kin, kout, Lout = dual_leg(FL->legs[2]), Lin = FL->legs[2];
    kin.dir = 1;
    kout.dir = -1;
    for (auto& c : secs)
        if (c.k > 0) { kin.q.push_back(c.key); kin.d.push_back(c.k); }
    kout.q = kin.q;
    kout.d = kin.d;
    P2->legs = {Lout, kin};
    Pt2->legs = {kout, Lin};
    for (auto* X : {P2.get(), Pt2.get()}) {
        X->group = SYMTEN_SU2;
        X->flux = 0;
        X->dtype = SYMTEN_F64;
        X->elems = po.ptot;
        X->meta_only = false;
    }
    P2->buf = po.P;
    Pt2->buf = po.Pt;
    for (auto& c : secs) {
        if (c.k == 0) continue;
        Block pb;
        pb.q = {c.key, c.key};
        pb.tree = {c.key};
        pb.shape = {c.n, c.k};
        pb.stride = {1, c.n};
        pb.offset = c.pbase;
        pb.size = (int64_t)c.n * c.k;
        P2->blocks.push_back(pb);
        Block tb = pb;
        tb.shape = {c.k, c.n};
        tb.stride = {1, c.k};
        Pt2->blocks.push_back(tb);
    }
    P2->rebuild_index();
    Pt2->rebuild_index();
    TensorPtr P2c = P2, Pt2c = Pt2;
    if (!f64) {
        P2c = std::make_shared<Tensor>(*P2);
        Pt2c = std::make_shared<Tensor>(*Pt2);
        P2c->dtype = Pt2c->dtype = SYMTEN_F32;
        P2c->buf = device_alloc(4 * std::max<int64_t>(po.ptot, 1));
        Pt2c->buf = device_alloc(4 * std::max<int64_t>(po.ptot, 1));
        launch_cast(P2->buf->ptr, true, P2c->buf->ptr, false, po.ptot, s);
        launch_cast(Pt2->buf->ptr, true, Pt2c->buf->ptr, false, po.ptot, s);
    }
    std::vector<Contracted> pp = contract_batched({{FL.get(), P2c.get(), {2}, {0}, {}},          // P  = [x4, d, k]
                                                   {Pt2c.get(), FLbar.get(), {1}, {2}, {}}},   // P~ = [k, x4, d]
                                                  prec, s);
    TensorPtr Pc = pp[0].t, Ptc = pp[1].t;
    tm.mark(s);
    // ---- renormalise, as in the U(1) move ---------------------------------
    std::vector<Contracted> r3 =
        contract_batched({{k1.step1.get(), Pc.get(), {0, 1}, {0, 1}, {1, 0}},      // C1' = [k, x1]
                          {k4.step1.get(), Ptc.get(), {0, 2}, {1, 2}, {}},         // C4' = [x3, k]
                          {Ptc.get(), &T4, {1}, {2}, {}}},                         // P~ T4 = [k_hi, u, y, l]
                         prec, s);
    Contracted &c1n = r3[0], &c4n = r3[1], &t4a = r3[2];
    Contracted xx = contract(*t4a.t, a, {1, 3}, {1, 0}, {}, prec, s);              // [k_hi, y, r, d]
    Contracted t4n = contract(*xx.t, *Pc, {1, 3}, {0, 1}, {2, 1, 0}, prec, s);     // [k_lo, r, k_hi]
    for (TensorPtr X : {c1n.t, t4n.t, c4n.t}) normalise_su2(*X, f64, s);
    tm.mark(s);
    env->C[0] = c1n.t;
    env->T[3] = t4n.t;
    env->C[3] = c4n.t;
    env->P.t = Pc;
    env->Pt.t = Ptc;
    env->svals = po.sv;
    if (st) {
        std::memset(st, 0, sizeof(*st));
        HIPCHK(hipStreamSynchronize(s));
        fill_cut_stats(st, secs, po);
        st->flops_corners = k1.info.useful_flops + k2.info.useful_flops + k3.info.useful_flops + k4.info.useful_flops;
        st->flops_halves = hh[0].plan->info.useful_flops + hh[1].plan->info.useful_flops;
        st->flops_renorm = c1n.plan->info.useful_flops + t4a.plan->info.useful_flops + xx.plan->info.useful_flops +
                           t4n.plan->info.useful_flops + c4n.plan->info.useful_flops;
        st->ms_corners = tm.ms(0, 1);
        st->ms_halves = tm.ms(1, 2);
        st->ms_proj = tm.ms(2, 3);
        st->ms_renorm = tm.ms(3, 4);
        st->ms_total = tm.ms(0, 4);
    }
}

}  // namespace
}  // namespace symten

namespace symten {
namespace {
// ------------------------------------------------ network turned a quarter
// U(1) leg reversal: direction and charges negated, block data unchanged
// (the addition rule keeps holding; the sectors of the leg reverse order).
TensorPtr flip_legs_u1(const TensorPtr& t, std::initializer_list<int> legs) {
    auto r = std::make_shared<Tensor>(*t);
    const int cm = charge_mod(t->group);
    for (int l : legs) {
        Leg& L = r->legs[l];
        L.dir = -L.dir;
        std::vector<std::pair<int, int>> secs;
        for (size_t k = 0; k < L.q.size(); ++k) secs.push_back({cnorm(-L.q[k], cm), L.d[k]});
        std::sort(secs.begin(), secs.end());
        L.q.clear();
        L.d.clear();
        for (auto& sd : secs) { L.q.push_back(sd.first); L.d.push_back(sd.second); }
        for (auto& b : r->blocks) b.q[l] = cnorm(-b.q[l], cm);
    }
    std::sort(r->blocks.begin(), r->blocks.end(), [](const Block& x, const Block& y) { return x.q < y.q; });
    r->rebuild_index();
    return r;
}

// Leg permutation (new leg j = old leg perm[j]); shares the buffer.
TensorPtr permute_legs(const TensorPtr& t, const std::vector<int>& perm) {
    auto r = std::make_shared<Tensor>(*t);
    const int R = t->rank();
    for (int j = 0; j < R; ++j) r->legs[j] = t->legs[perm[j]];
    for (size_t i = 0; i < t->blocks.size(); ++i) {
        const Block& b = t->blocks[i];
        Block& nb = r->blocks[i];
        for (int j = 0; j < R; ++j) {
            nb.q[j] = b.q[perm[j]];
            nb.shape[j] = b.shape[perm[j]];
            nb.stride[j] = b.stride[perm[j]];
        }
    }
    std::sort(r->blocks.begin(), r->blocks.end(), [](const Block& x, const Block& y) { return x.q < y.q; });
    r->rebuild_index();
    return r;
}

// The network turned a quarter counterclockwise, in the conventions of the
// left move: C1' = C2, C2' = C3, C3' = C4, C4' = C1 and T1' = T2, T2' = T3,
// T3' = T4, T4' = T1 keep the clockwise chi bonds; a'[l,u,r,d] = a[u,r,d,l].
// The legs that land on the wrong side of the (in, in, out, out) convention
// of a, and the D^2 legs of T1' and T3', are reversed (both ends of each such
// bond).  Four turns give back the original tensors.
void rotate_ccw(std::array<TensorPtr, 4>& C, std::array<TensorPtr, 4>& T, TensorPtr& a) {
    const std::array<TensorPtr, 4> Cn{C[1], C[2], C[3], C[0]};
    const std::array<TensorPtr, 4> Tn{flip_legs_u1(T[1], {1}), T[2], flip_legs_u1(T[3], {1}), T[0]};
    a = flip_legs_u1(permute_legs(a, {1, 2, 3, 0}), {1, 3});
    C = Cn;
    T = Tn;
}

// Full trace of a rank-2 tensor whose two legs are the two ends of one bond
// (FP64 on the host).  An SU(2) block of spin j stands for its reduced
// matrix times the identity on the 2j+1 states of the multiplet (the basis
// tensor of one incoming and one outgoing leg of spin j), so its trace
// counts 2j+1 times.
double trace_bond(const Tensor& X) {
    if (X.rank() != 2) fail(SYMTEN_E_INVAL, "internal: trace of a non-matrix");
    std::vector<char> host((size_t)std::max<int64_t>(X.elems, 1) * X.esize());
    HIPCHK(hipMemcpy(host.data(), X.data(), X.elems * X.esize(), hipMemcpyDeviceToHost));
    double t = 0.0;
    for (const Block& b : X.blocks) {
        if (b.q[0] != b.q[1] || b.shape[0] != b.shape[1]) continue;
        const double mult = X.group == SYMTEN_SU2 ? (double)(b.q[0] + 1) : 1.0;
        for (int i = 0; i < b.shape[0]; ++i) {
            const int64_t o = b.offset + i * (b.stride[0] + b.stride[1]);
            t += mult * (X.dtype == SYMTEN_F64 ? ((const double*)host.data())[o]
                                               : (double)((const float*)host.data())[o]);
        }
    }
    return t;
}

// FP64 copy of a tensor (same blocks and strides).
TensorPtr as_f64(const TensorPtr& t, hipStream_t s) {
    if (t->dtype == SYMTEN_F64) return t;
    auto r = std::make_shared<Tensor>(*t);
    r->dtype = SYMTEN_F64;
    r->buf = device_alloc(8 * std::max<int64_t>(t->elems, 1));
    launch_cast(t->data(), false, r->buf->ptr, true, t->elems, s);
    return r;
}

// A tensor of a closed network with one bond label per leg.
struct Labelled {
    TensorPtr t;
    std::vector<int> lab;
};

// X contracted with Y over every bond label they share except `keep` (the
// bond left open for the closing trace), in FP64; the result's legs are X's
// open legs in order, then Y's.
Labelled join(const Labelled& X, const Labelled& Y, int keep, hipStream_t s) {
    std::vector<int> la, lb;
    for (size_t i = 0; i < X.lab.size(); ++i)
        for (size_t j = 0; j < Y.lab.size(); ++j)
            if (X.lab[i] == Y.lab[j] && X.lab[i] != keep) {
                la.push_back((int)i);
                lb.push_back((int)j);
            }
    if (la.empty()) fail(SYMTEN_E_INVAL, "internal: network step without a shared bond");
    auto p = get_plan(*X.t, *Y.t, (int)la.size(), la.data(), lb.data(), nullptr, SYMTEN_PREC_F64);
    Labelled r{run_contraction(*p, *X.t, *Y.t, s), {}};
    for (size_t i = 0; i < X.lab.size(); ++i)
        if (std::find(la.begin(), la.end(), (int)i) == la.end()) r.lab.push_back(X.lab[i]);
    for (size_t j = 0; j < Y.lab.size(); ++j)
        if (std::find(lb.begin(), lb.end(), (int)j) == lb.end()) r.lab.push_back(Y.lab[j]);
    return r;
}

// Z_nm: the four corners with n columns and m rows of edge tensors between
// them and the n x m site tensors a inside (n, m <= 2), contracted in FP64.
// Bonds: the chi bonds run C1 -h-> T1 .. T1 -> C2 -v-> T2 .. T2 -> C3 -g->
// T3 (right to left) -> C4 -w-> T4 (bottom to top) -> C1; the D bonds are
// vert(i, j) below row i of column j (row 0 = the T1 row) and hor(i, j) right
// of column j in row i (column 0 = the T4 column).  C1's incoming bond stays
// open until the end and closes as a trace.
// sites (optional): n*m tensors replacing a, row i (top to bottom) major,
// column j (left to right) minor.
double zblock(const std::array<TensorPtr, 4>& C, const std::array<TensorPtr, 4>& T, const TensorPtr& a, int n,
              int m, hipStream_t s, const TensorPtr* sites = nullptr) {
    auto h = [](int j) { return 1000 + j; };
    auto v = [](int i) { return 2000 + i; };
    auto g = [](int j) { return 3000 + j; };
    auto w = [](int i) { return 4000 + i; };
    auto vert = [](int i, int j) { return 5000 + 100 * i + j; };
    auto hor = [](int i, int j) { return 6000 + 100 * i + j; };
    const int keep = w(m);
    Labelled X{C[0], {w(m), h(0)}};
    for (int j = 1; j <= n; ++j) X = join(X, {T[0], {h(j - 1), vert(0, j), h(j)}}, keep, s);
    X = join(X, {C[1], {h(n), v(0)}}, keep, s);
    for (int i = 1; i <= m; ++i) {
        X = join(X, {T[1], {v(i - 1), hor(i, n), v(i)}}, keep, s);
        for (int j = n; j >= 1; --j) {
            const TensorPtr& site = sites ? sites[(i - 1) * n + (j - 1)] : a;
            X = join(X, {site, {hor(i, j - 1), vert(i - 1, j), hor(i, j), vert(i, j)}}, keep, s);
        }
        X = join(X, {T[3], {w(m - i), hor(i, 0), w(m - i + 1)}}, keep, s);
    }
    X = join(X, {C[2], {v(m), g(0)}}, keep, s);
    for (int j = n; j >= 1; --j) X = join(X, {T[2], {g(n - j), vert(m, j), g(n - j + 1)}}, keep, s);
    X = join(X, {C[3], {g(n), w(0)}}, keep, s);
    if (X.t->rank() != 2 || X.lab[0] != keep || X.lab[1] != keep) fail(SYMTEN_E_INVAL, "internal: network not closed");
    return trace_bond(*X.t);
}

// Partition function per site of a classical model from the environment of a
// 1x1 cell, estimated on a b x b block: kappa^(b^2) = Z_bb Z_00 / (Z_b0 Z_0b),
// the boundary factors cancelling in the ratio.  b = 2 also cancels the
// corner weights when the environment bonds alternate between two charge
// parities from one site to the next (every D charge odd): with one column or
// row the corners of the two parity copies pair up unequally.  z receives
// Z_00, Z_b0, Z_0b, Z_bb.
double site_partition(ctm_env* env, const TensorPtr& a_in, int b, double z[4], hipStream_t s) {
    std::array<TensorPtr, 4> C, T;
    for (int i = 0; i < 4; ++i) {
        C[i] = as_f64(env->C[i], s);
        T[i] = as_f64(env->T[i], s);
    }
    TensorPtr a = as_f64(a_in, s);
    z[0] = zblock(C, T, a, 0, 0, s);
    z[1] = zblock(C, T, a, b, 0, s);
    z[2] = zblock(C, T, a, 0, b, s);
    z[3] = zblock(C, T, a, b, b, s);
    const double den = z[1] * z[2];
    if (den == 0.0 || !std::isfinite(den)) fail(SYMTEN_E_LINALG, "site partition: vanishing normalisation");
    const double r = z[3] * z[0] / den;
    if (b == 1) return r;
    if (!(r > 0.0)) fail(SYMTEN_E_LINALG, "site partition: non-positive block ratio");
    return std::pow(r, 1.0 / (b * b));
}

std::array<TensorPtr, 4> env_f64(const TensorPtr* X, hipStream_t s) {
    std::array<TensorPtr, 4> r;
    for (int i = 0; i < 4; ++i) r[i] = as_f64(X[i], s);
    return r;
}

// <O> = Z_nm(sites) / Z_nm(a): the n x m patch with its site tensors replaced
// (row-major), in FP64.
double expectation(ctm_env* env, const TensorPtr& a, int n, int m, const std::vector<TensorPtr>& sites,
                   hipStream_t s) {
    std::array<TensorPtr, 4> C = env_f64(env->C, s), T = env_f64(env->T, s);
    TensorPtr a64 = as_f64(a, s);
    std::vector<TensorPtr> b;
    for (const auto& x : sites) b.push_back(as_f64(x, s));
    const double z = zblock(C, T, a64, n, m, s);
    if (z == 0.0 || !std::isfinite(z)) fail(SYMTEN_E_LINALG, "expectation: vanishing normalisation");
    return zblock(C, T, a64, n, m, s, b.data()) / z;
}
}  // namespace
}  // namespace symten

namespace symten {
namespace {
// One U(1) left move on the environment's current tensors (see ctm_move).
// The projectors of one horizontal cut from the four enlarged corners
// around it (the halves H_u = C~1 C~2, H_d = C~4 C~3, then the FP64 stage):
// P[chi out, D in, k in] below the upper half, P~[k out, chi in, D out]
// above the lower half; chiL and dL are the chi and D legs of the cut (the
// lower legs of C~1).  Pc, Ptc: the same in the storage precision.
struct CutResult {
    TensorPtr P, Pt, Pc, Ptc;
    ProjOut po;
    std::vector<CutSector> secs;
    std::vector<Contracted> halves;
};
// A cut up to its eigensolves: the halves and the sector matrices H_u^T,
// H_d^T over the union of their row blocks.
struct CutPrep {
    CutResult cr;
    std::vector<CutSector> secs;
    std::map<int, std::vector<std::vector<int>>> rows_of;      // Q -> union rows
    std::map<int, std::map<std::vector<int>, int>> row_off_of;
    std::vector<BufferPtr> row_bufs;                           // read by the solves
    Leg chiL, dL;
    int group = 0;
    bool f64 = false;
};
CutPrep cut_prepare(const CornerResult& k1, const CornerResult& k2, const CornerResult& k3, const CornerResult& k4,
                    const Leg& chiL, const Leg& dL, int group, int prec, Timer* tm, hipStream_t s) {
    const bool f64 = prec == SYMTEN_PREC_F64;
    CutPrep cp;
    CutResult& cr = cp.cr;
    // halves: H_u = C~1 C~2 -> [x4, d, x2, d2]; H_d = C~4 C~3 -> [x4, u, x2, u3]
    cr.halves = contract_batched({{k1.corner.get(), k2.corner.get(), {0, 2}, {0, 2}, {}},
                                  {k4.corner.get(), k3.corner.get(), {0, 3}, {0, 2}, {}}},
                                 prec, s);
    Contracted &hu = cr.halves[0], &hd = cr.halves[1];
    if (tm) tm->mark(s);
    // ---- projectors, per fused charge Q of the left cut (FP64) ----------
    std::map<int, const GroupPlan*> gu_of, gd_of;
    const int cm = charge_mod(group);
    for (auto& g : hu.plan->groups) gu_of[cnorm(g.rows[0][0] - g.rows[0][1], cm)] = &g;
    for (auto& g : hd.plan->groups) gd_of[cnorm(g.rows[0][0] - g.rows[0][1], cm)] = &g;
    const size_t es = f64 ? 8 : 4;
    // The rows of both halves are the (q_chi, q_D) blocks of the cut reached
    // by their contractions; where the two sets differ, both halves are laid
    // out over the union (rows missing on one side are zero).
    std::vector<CutSector> secs;
    std::map<int, std::vector<std::vector<int>>> rows_of;   // Q -> union rows
    std::map<int, std::map<std::vector<int>, int>> row_off_of;
    std::vector<BufferPtr> row_bufs;
    std::vector<CopyTask> row_tasks[2];
    int64_t row_elems[2] = {0, 0};
    struct Pending { size_t sec; int side; int64_t off; };
    std::vector<Pending> pending;
    for (auto& kv : gu_of) {
        auto it = gd_of.find(kv.first);
        if (it == gd_of.end()) continue;   // no weight on one side: nothing to keep
        const GroupPlan* gs[2] = {kv.second, it->second};
        std::vector<std::vector<int>> rows = gs[0]->rows;
        rows.insert(rows.end(), gs[1]->rows.begin(), gs[1]->rows.end());
        std::sort(rows.begin(), rows.end());
        rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
        std::map<std::vector<int>, int> roff;
        int n = 0;
        for (auto& r : rows) {
            roff[r] = n;
            n += chiL.dim_of(r[0]) * dL.dim_of(r[1]);
        }
        CutSector c;
        c.key = kv.first;
        c.weight = 1;
        c.n = n;
        c.mu = gs[0]->N;
        c.md = gs[1]->N;
        for (int side = 0; side < 2; ++side) {
            const GroupPlan* g = gs[side];
            const Tensor& H = side == 0 ? *hu.t : *hd.t;
            const void* base = (const char*)H.data() + g->c_off * es;
            if (g->rows == rows) {
                (side == 0 ? c.hu : c.hd) = base;
                continue;
            }
            // copy the present row blocks into a zeroed union-row matrix
            const int m = g->N;
            for (size_t r = 0; r < g->rows.size(); ++r) {
                const int rd = chiL.dim_of(g->rows[r][0]) * dL.dim_of(g->rows[r][1]);
                row_tasks[side].push_back(make_copy_task(0, g->c_off + (int64_t)g->row_off[r] * m, 1,
                                                         row_elems[side] + (int64_t)roff[g->rows[r]] * m,
                                                         {rd, m}, {m, 1}, {m, 1}));
                row_tasks[side].back().src_buf = side;   // 0: H_u, 1: H_d
                row_tasks[side].back().dst_buf = 2 + side;
            }
            pending.push_back({secs.size(), side, row_elems[side]});
            row_elems[side] += (int64_t)n * m;
        }
        rows_of[c.key] = rows;
        row_off_of[c.key] = roff;
        secs.push_back(c);
    }
    if (!pending.empty()) {
        BufferPtr ub[2];
        for (int side = 0; side < 2; ++side) {
            ub[side] = device_alloc(std::max<int64_t>(row_elems[side], 1) * es);
            launch_fill_zero(ub[side]->ptr, ((std::max<int64_t>(row_elems[side], 1) * es + 3) / 4) * 4, s);
            row_bufs.push_back(ub[side]);
        }
        std::vector<CopyTask> tasks = row_tasks[0];
        tasks.insert(tasks.end(), row_tasks[1].begin(), row_tasks[1].end());
        validate_tasks(tasks, {hu.t->elems, hd.t->elems, std::max<int64_t>(row_elems[0], 1),
                               std::max<int64_t>(row_elems[1], 1)});
        std::vector<int64_t> prefix;
        copy_prefix(tasks, prefix);
        BufferPtr dt, dp;
        upload_sync(dt, tasks.data(), tasks.size() * sizeof(CopyTask));
        upload_sync(dp, prefix.data(), prefix.size() * sizeof(int64_t));
        copy_launch_arg((const CopyTask*)dt->ptr, (const int64_t*)dp->ptr, (int)tasks.size(), prefix.back(),
                        {hu.t->data(), hd.t->data(), ub[0]->ptr, ub[1]->ptr}, f64, f64 ? 1 : 0, s);
        row_bufs.push_back(dt);
        row_bufs.push_back(dp);
        for (auto& pd : pending)
            (pd.side == 0 ? secs[pd.sec].hu : secs[pd.sec].hd) = (const char*)ub[pd.side]->ptr + pd.off * es;
    }
    cp.secs = std::move(secs);
    cp.rows_of = std::move(rows_of);
    cp.row_off_of = std::move(row_off_of);
    cp.row_bufs = std::move(row_bufs);
    cp.chiL = chiL;
    cp.dL = dL;
    cp.group = group;
    cp.f64 = f64;
    return cp;
}

// The projector tensors of a prepared cut whose eigensolves are finished.
CutResult cut_complete(CutPrep& cp, const ProjOut& po, hipStream_t s) {
    CutResult& cr = cp.cr;
    std::vector<CutSector>& secs = cp.secs;
    auto& rows_of = cp.rows_of;
    auto& row_off_of = cp.row_off_of;
    const Leg &chiL = cp.chiL, &dL = cp.dL;
    const int group = cp.group;
    const bool f64 = cp.f64;
    // ---- projector tensors P[chi out, D in, k in], P~[k out, chi in, D out]
    auto P = std::make_shared<Tensor>();
    auto Pt = std::make_shared<Tensor>();
    for (auto* X : {P.get(), Pt.get()}) {
        X->group = group;
        X->flux = 0;
        X->dtype = SYMTEN_F64;
    }
    Leg kin, kout;
    kin.dir = 1;
    kout.dir = -1;
    for (auto& c : secs)
        if (c.k > 0) { kin.q.push_back(c.key); kin.d.push_back(c.k); }
    kout.q = kin.q;
    kout.d = kin.d;
    Leg chi_out = chiL, chi_in = chiL, d_in = dL, d_out = dL;
    chi_out.dir = -1;
    chi_in.dir = 1;
    d_in.dir = 1;
    d_out.dir = -1;
    P->legs = {chi_out, d_in, kin};
    Pt->legs = {kout, chi_in, d_out};
    const int64_t ptot = po.ptot;
    P->buf = po.P;
    Pt->buf = po.Pt;
    P->elems = Pt->elems = ptot;
    P->meta_only = Pt->meta_only = false;
    for (auto& c : secs) {
        if (c.k == 0) continue;
        const int Q = c.key, n = c.n, k = c.k;
        // blocks: one per (q_chi, q_D) row sub-block of this sector
        for (const auto& row : rows_of[Q]) {
            const int qx = row[0], qd = row[1];
            const int dx = chiL.dim_of(qx), dd = dL.dim_of(qd);
            const int64_t ro = row_off_of[Q][row];
            Block pb;
            pb.q = {qx, qd, Q};
            pb.shape = {dx, dd, k};
            pb.stride = {dd, 1, n};
            pb.offset = c.pbase + ro;
            pb.size = (int64_t)dx * dd * k;
            P->blocks.push_back(pb);
            Block tb;
            tb.q = {Q, qx, qd};
            tb.shape = {k, dx, dd};
            tb.stride = {1, (int64_t)dd * k, k};
            tb.offset = c.pbase + ro * k;
            tb.size = pb.size;
            Pt->blocks.push_back(tb);
        }
    }
    for (auto* X : {P.get(), Pt.get()}) {
        std::sort(X->blocks.begin(), X->blocks.end(), [](const Block& x, const Block& y) { return x.q < y.q; });
        X->rebuild_index();
    }
    TensorPtr Pc = P, Ptc = Pt;
    if (!f64) {
        Pc = std::make_shared<Tensor>(*P);
        Ptc = std::make_shared<Tensor>(*Pt);
        Pc->dtype = Ptc->dtype = SYMTEN_F32;
        Pc->buf = device_alloc(4 * std::max<int64_t>(ptot, 1));
        Ptc->buf = device_alloc(4 * std::max<int64_t>(ptot, 1));
        launch_cast(P->buf->ptr, true, Pc->buf->ptr, false, ptot, s);
        launch_cast(Pt->buf->ptr, true, Ptc->buf->ptr, false, ptot, s);
    }
    cr.P = P;
    cr.Pt = Pt;
    cr.Pc = Pc;
    cr.Ptc = Ptc;
    cr.po = po;
    cr.secs = secs;
    return cr;
}

CutResult cut_from_corners(ctm_env* env, const CornerResult& k1, const CornerResult& k2, const CornerResult& k3,
                           const CornerResult& k4, const Leg& chiL, const Leg& dL, int group, int chi, int prec,
                           Timer* tm, hipStream_t s) {
    CutPrep cp = cut_prepare(k1, k2, k3, k4, chiL, dL, group, prec, tm, s);
    ProjOut po = cut_projectors(env, cp.secs, chi, cp.f64, s);
    return cut_complete(cp, po, s);
}

// C1' = (C1 T1) P_above, T4' = P~_above (T4 a) P_below, C4' = (C4 T3) P~_below^T,
// each scaled to unit Frobenius norm in FP64; c1t1 and c4t3 are the first
// steps of enlarged corners 1 and 4 (C1 T1 and C4 T3).
struct Renormalised {
    TensorPtr C1, T4, C4;
    symten_plan_stats info{};
};
Renormalised renormalise_left(const Tensor& c1t1, const Tensor& c4t3, const Tensor& T4, const Tensor& a,
                              const CutResult& above, const CutResult& below, int prec, hipStream_t s) {
    const bool f64 = prec == SYMTEN_PREC_F64;
    // T4' = ((P~ T4) a) P: absorbing P~ first keeps the intermediates at
    // chi' chi D^4 instead of the chi^2 D^6 of T4 a.
    std::vector<Contracted> r3 =
        contract_batched({{&c1t1, above.Pc.get(), {0, 1}, {0, 1}, {1, 0}},      // C1' = [k, x1]
                          {&c4t3, below.Ptc.get(), {0, 2}, {1, 2}, {}},         // C4' = [x3, k]
                          {above.Ptc.get(), &T4, {1}, {2}, {}}},                // P~ T4 = [k_hi, u, y, l]
                         prec, s);
    Contracted &c1n = r3[0], &c4n = r3[1], &t4a = r3[2];
    Contracted xx = contract(*t4a.t, a, {1, 3}, {1, 0}, {}, prec, s);               // [k_hi, y, r, d]
    Contracted t4n = contract(*xx.t, *below.Pc, {1, 3}, {0, 1}, {2, 1, 0}, prec, s);  // [k_lo, r, k_hi]
    BufferPtr red = device_alloc(8 * (1 + 512));
    for (TensorPtr X : {c1n.t, t4n.t, c4n.t}) {
        launch_sumsq(X->data(), f64, X->elems, (double*)red->ptr, s);
        launch_scale_by_inv_sqrt(X->data(), f64, X->elems, (const double*)red->ptr, s);
    }
    Renormalised r;
    r.C1 = c1n.t;
    r.T4 = t4n.t;
    r.C4 = c4n.t;
    for (auto* c : {&c1n, &t4a, &xx, &t4n, &c4n}) add_info(r.info, c->plan->info);
    return r;
}

void move_u1_left(ctm_env* env, Tensor& a, int chi, int prec, ctm_move_stats* st, hipStream_t s) {
    Timer tm;
    tm.init(st != nullptr);
    tm.mark(s);
    Tensor &C1 = *env->C[0], &C2 = *env->C[1], &C3 = *env->C[2], &C4 = *env->C[3];
    Tensor &T1 = *env->T[0], &T2 = *env->T[1], &T3 = *env->T[2], &T4 = *env->T[3];
    // the four corners are independent: each of their three steps is one
    // gather launch and one grouped-GEMM launch for all four
    std::vector<CornerResult> ks =
        corners_batched({1, 2, 3, 4}, {{&C1, &T1, &T4}, {&C2, &T1, &T2}, {&C3, &T3, &T2}, {&C4, &T3, &T4}}, a,
                        prec, s);
    CornerResult &k1 = ks[0], &k2 = ks[1], &k3 = ks[2], &k4 = ks[3];
    tm.mark(s);
    CutResult cr = cut_from_corners(env, k1, k2, k3, k4, T4.legs[0], a.legs[3], a.group, chi, prec, &tm, s);
    tm.mark(s);
    // ---- renormalise (one cut above and below: the 1x1 cell) ------------
    Renormalised rn = renormalise_left(*k1.step1, *k4.step1, T4, a, cr, cr, prec, s);
    tm.mark(s);
    env->C[0] = rn.C1;
    env->T[3] = rn.T4;
    env->C[3] = rn.C4;
    env->P.t = cr.P;
    env->Pt.t = cr.Pt;
    env->svals = cr.po.sv;
    if (st) {
        std::memset(st, 0, sizeof(*st));
        HIPCHK(hipStreamSynchronize(s));
        fill_cut_stats(st, cr.secs, cr.po);
        st->flops_corners = k1.info.useful_flops + k2.info.useful_flops + k3.info.useful_flops + k4.info.useful_flops;
        st->flops_halves = cr.halves[0].plan->info.useful_flops + cr.halves[1].plan->info.useful_flops;
        st->flops_renorm = rn.info.useful_flops;

        st->ms_corners = tm.ms(0, 1);
        st->ms_halves = tm.ms(1, 2);
        st->ms_proj = tm.ms(2, 3);
        st->ms_renorm = tm.ms(3, 4);
        st->ms_total = tm.ms(0, 4);
    }
}

// Left move of a unit cell, column by column (x = 0 .. Lx-1): the projectors
// of every cut y (between site rows y and y+1) from the 2 x 2 block of sites
// (x, y) .. (x+1, y+1), each site's enlarged corner built from its own
// environment, then the left column of the sites (x+1, y):
// C1' = P(y-1)^T C1 T1 (x, y), T4' = P~(y-1) T4 a (x, y) P(y),
// C4' = C4 T3 (x, y) P~(y)^T.  Column x+1 is updated before column x+1 is
// used (the moves run one after another).  a[x Ly + y] are the site tensors.
void cell_left_move(ctm_env* env, const std::vector<TensorPtr>& a, int chi, int prec, hipStream_t s) {
    const int Lx = env->Lx, Ly = env->Ly;
    auto C = [&](int x, int y, int i) -> Tensor& { return *env->cC[4 * (((x % Lx) + Lx) % Lx * Ly + ((y % Ly) + Ly) % Ly) + i]; };
    auto T = [&](int x, int y, int i) -> Tensor& { return *env->cT[4 * (((x % Lx) + Lx) % Lx * Ly + ((y % Ly) + Ly) % Ly) + i]; };
    auto A = [&](int x, int y) -> Tensor& { return *a[((x % Lx) + Lx) % Lx * Ly + ((y % Ly) + Ly) % Ly]; };
    env->svals.clear();
    for (int x = 0; x < Lx; ++x) {
        const int x1 = x + 1;
        std::vector<CutResult> cuts(Ly);
        std::vector<CutPrep> preps(Ly);
        std::vector<TensorPtr> c1t1(Ly), c4t3(Ly);
        for (int y = 0; y < Ly; ++y) {
            const int y1 = y + 1;
            std::vector<const Tensor*> as = {&A(x, y), &A(x1, y), &A(x1, y1), &A(x, y1)};
            std::vector<CornerResult> ks = corners_batched(
                {1, 2, 3, 4},
                {{&C(x, y, 0), &T(x, y, 0), &T(x, y, 3)}, {&C(x1, y, 1), &T(x1, y, 0), &T(x1, y, 1)},
                 {&C(x1, y1, 2), &T(x1, y1, 2), &T(x1, y1, 1)}, {&C(x, y1, 3), &T(x, y1, 2), &T(x, y1, 3)}},
                A(x, y), prec, s, &as);
            preps[y] = cut_prepare(ks[0], ks[1], ks[2], ks[3], T(x, y, 3).legs[0], A(x, y).legs[3], A(x, y).group,
                                   prec, nullptr, s);
            c1t1[y] = ks[0].step1;             // C1 T1 of site (x, y)
            c4t3[y1 % Ly] = ks[3].step1;       // C4 T3 of site (x, y+1)
        }
        // the cuts of a column are independent: their eigensolves are all
        // enqueued before the first read-back, spread over the streams
        HIPCHK(hipEventRecord(env->ev_start, s));
        std::vector<std::vector<CutSector>*> cut_secs;
        for (int y = 0; y < Ly; ++y) cut_secs.push_back(&preps[y].secs);
        std::vector<ProjPending> pend = issue_solves(env, cut_secs, preps[0].f64, s, env->ev_start);
        for (int y = 0; y < Ly; ++y) {
            ProjOut po = finish_projectors(env, preps[y].secs, pend[y], chi, preps[y].f64, s);
            cuts[y] = cut_complete(preps[y], po, s);
            // the kept values of the cut, descending
            std::vector<double> sv = cuts[y].po.sv;
            std::sort(sv.begin(), sv.end(), std::greater<double>());
            int kept = 0;
            for (auto& c : cuts[y].secs) kept += c.k * c.weight;
            env->svals.insert(env->svals.end(), sv.begin(), sv.begin() + std::min<size_t>(kept, sv.size()));
        }
        std::vector<Renormalised> rn;
        for (int y = 0; y < Ly; ++y)
            rn.push_back(renormalise_left(*c1t1[y], *c4t3[y], T(x, y, 3), A(x, y), cuts[(y + Ly - 1) % Ly], cuts[y],
                                          prec, s));
        const int xn = x1 % Lx;
        for (int y = 0; y < Ly; ++y) {
            env->cC[4 * (xn * Ly + y) + 0] = rn[y].C1;
            env->cT[4 * (xn * Ly + y) + 3] = rn[y].T4;
            env->cC[4 * (xn * Ly + y) + 3] = rn[y].C4;
        }
        env->P.t = cuts[Ly - 1].P;
        env->Pt.t = cuts[Ly - 1].Pt;
    }
}
}  // namespace
}  // namespace symten

// =================================================================== C ABI
extern "C" {

const char* symten_last_error(void) { return g_err.c_str(); }
int symten_version(void) { return 1; }

int symten_sync(void* stream) {
    return guard_on(stream, [&] { HIPCHK(hipStreamSynchronize(S(stream))); });
}

int symten_create_meta(symten_t* out, const symten_desc* d) {
    return guard([&] {
        if (!out) fail(SYMTEN_E_INVAL, "null output");
        *out = wrap(make_desc_tensor(d));
    });
}

int symten_create(symten_t* out, const symten_desc* d, void* stream) {
    return guard_on(stream, [&] {
        if (!out) fail(SYMTEN_E_INVAL, "null output");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
            (void)hipGetLastError();
            fail(SYMTEN_E_NODEVICE, "no GPU available");
        }
        auto t = make_desc_tensor(d);
        t->buf = device_alloc(std::max<int64_t>(t->elems, 1) * t->esize());
        t->meta_only = false;
        launch_fill_zero(t->buf->ptr, ((std::max<int64_t>(t->elems, 1) * t->esize() + 3) / 4) * 4, S(stream));
        *out = wrap(t);
    });
}

void symten_destroy(symten_t t) { delete t; }

int symten_rank(symten_t t, int* r) {
    return guard([&] { if (!r) fail(SYMTEN_E_INVAL, "null"); *r = T(t).rank(); });
}
int symten_flux(symten_t t, int* f) {
    return guard([&] { if (!f) fail(SYMTEN_E_INVAL, "null"); *f = T(t).flux; });
}
int symten_dtype(symten_t t, int* d) {
    return guard([&] { if (!d) fail(SYMTEN_E_INVAL, "null"); *d = T(t).dtype; });
}
int symten_leg_info(symten_t t, int leg, int* dir, int* nsec, int* labels, int* dims) {
    return guard([&] {
        Tensor& x = T(t);
        if (leg < 0 || leg >= x.rank()) fail(SYMTEN_E_INVAL, "leg out of range");
        const Leg& L = x.legs[leg];
        if (dir) *dir = L.dir;
        if (nsec) *nsec = (int)L.q.size();
        for (size_t i = 0; i < L.q.size(); ++i) {
            if (labels) labels[i] = L.q[i];
            if (dims) dims[i] = L.d[i];
        }
    });
}
int symten_num_blocks(symten_t t, int64_t* n) {
    return guard([&] { if (!n) fail(SYMTEN_E_INVAL, "null"); *n = (int64_t)T(t).blocks.size(); });
}
int symten_nnz(symten_t t, int64_t* n) {
    return guard([&] { if (!n) fail(SYMTEN_E_INVAL, "null"); *n = T(t).nnz(); });
}
int symten_block_info(symten_t t, int64_t i, int* labels, int* shape, int64_t* offset, int64_t* strides) {
    return guard([&] {
        Tensor& x = T(t);
        if (i < 0 || i >= (int64_t)x.blocks.size()) fail(SYMTEN_E_INVAL, "block index out of range");
        const Block& b = x.blocks[i];
        for (int l = 0; l < x.rank(); ++l) {
            if (labels) labels[l] = b.q[l];
            if (shape) shape[l] = b.shape[l];
            if (strides) strides[l] = b.stride[l];
        }
        if (offset) *offset = b.offset;
    });
}
int symten_block_tree(symten_t t, int64_t i, int* ntree, int* tree) {
    return guard([&] {
        Tensor& x = T(t);
        if (i < 0 || i >= (int64_t)x.blocks.size()) fail(SYMTEN_E_INVAL, "block index out of range");
        const Block& b = x.blocks[i];
        if (ntree) *ntree = (int)b.tree.size();
        if (tree)
            for (size_t k = 0; k < b.tree.size(); ++k) tree[k] = b.tree[k];
    });
}
int symten_su2_to_u1(symten_t* out, symten_t in, void* stream) {
    return guard_on(stream, [&] {
        if (!out) fail(SYMTEN_E_INVAL, "null output");
        *out = wrap(su2_to_u1(T(in), S(stream)));
    });
}
int symten_su2_cg(int tj1, int tm1, int tj2, int tm2, int tJ, int tM, double* value) {
    return guard([&] {
        if (!value) fail(SYMTEN_E_INVAL, "null output");
        if (tj1 < 0 || tj2 < 0 || tJ < 0 || tj1 > 64 || tj2 > 64 || tJ > 128)
            fail(SYMTEN_E_INVAL, "doubled spins must be 0..64 (J: 0..128)");
        *value = cg_coeff(tj1, tm1, tj2, tm2, tJ, tM);
    });
}
int symten_set_allocator(void* (*alloc)(size_t, void*), void (*free_fn)(void*, size_t, void*), void* ctx) {
    return guard([&] {
        if ((alloc == nullptr) != (free_fn == nullptr)) fail(SYMTEN_E_INVAL, "allocator and free come as a pair");
        set_user_allocator(alloc, free_fn, ctx);
    });
}

int symten_nbytes(symten_t t, int64_t* bytes) {
    return guard([&] {
        if (!bytes) fail(SYMTEN_E_INVAL, "null output");
        Tensor& x = T(t);
        *bytes = x.elems * (int64_t)x.esize();
    });
}

int symten_device_ptr(symten_t t, void** ptr, int64_t* elems) {
    return guard([&] {
        Tensor& x = T(t);
        if (ptr) *ptr = x.data();
        if (elems) *elems = x.elems;
    });
}

int symten_upload(symten_t t, const double* values, int64_t n, void* stream) {
    return guard_on(stream, [&] {
        Tensor& x = T(t);
        check_device_tensor(x, "upload");
        if (n != x.nnz()) fail(SYMTEN_E_INVAL, "upload: value count differs from nnz");
        if (n > 0 && !values) fail(SYMTEN_E_INVAL, "upload: null values");
        const size_t es = x.esize();
        std::vector<char> host((size_t)std::max<int64_t>(x.elems, 1) * es, 0);
        HIPCHK(hipStreamSynchronize(S(stream)));
        HIPCHK(hipMemcpy(host.data(), x.data(), x.elems * es, hipMemcpyDeviceToHost));
        int64_t pos = 0;
        for (auto& b : x.blocks) {
            const int R = x.rank();
            std::vector<int> idx(R, 0);
            for (int64_t e = 0; e < b.size; ++e) {
                int64_t off = b.offset;
                for (int l = 0; l < R; ++l) off += idx[l] * b.stride[l];
                const double v = values[pos++];
                if (x.dtype == SYMTEN_F64) ((double*)host.data())[off] = v;
                else ((float*)host.data())[off] = (float)v;
                for (int l = R - 1; l >= 0; --l) {
                    if (++idx[l] < b.shape[l]) break;
                    idx[l] = 0;
                }
            }
        }
        HIPCHK(hipMemcpy(x.data(), host.data(), x.elems * es, hipMemcpyHostToDevice));
    });
}

int symten_download(symten_t t, double* values, int64_t n, void* stream) {
    return guard_on(stream, [&] {
        Tensor& x = T(t);
        check_device_tensor(x, "download");
        if (n != x.nnz()) fail(SYMTEN_E_INVAL, "download: value count differs from nnz");
        if (n > 0 && !values) fail(SYMTEN_E_INVAL, "download: null values");
        const size_t es = x.esize();
        std::vector<char> host((size_t)std::max<int64_t>(x.elems, 1) * es, 0);
        HIPCHK(hipStreamSynchronize(S(stream)));
        HIPCHK(hipMemcpy(host.data(), x.data(), x.elems * es, hipMemcpyDeviceToHost));
        int64_t pos = 0;
        for (auto& b : x.blocks) {
            const int R = x.rank();
            std::vector<int> idx(R, 0);
            for (int64_t e = 0; e < b.size; ++e) {
                int64_t off = b.offset;
                for (int l = 0; l < R; ++l) off += idx[l] * b.stride[l];
                values[pos++] = x.dtype == SYMTEN_F64 ? ((double*)host.data())[off] : (double)((float*)host.data())[off];
                for (int l = R - 1; l >= 0; --l) {
                    if (++idx[l] < b.shape[l]) break;
                    idx[l] = 0;
                }
            }
        }
    });
}

int symten_plan_info(symten_t A, symten_t B, int ncon, const int* legsA, const int* legsB, const int* out_perm,
                     symten_plan_stats* info, symten_t* out) {
    return guard([&] {
        auto p = plan_contraction(T(A), T(B), ncon, legsA, legsB, out_perm, T(A).dtype == SYMTEN_F64 ? SYMTEN_PREC_F64 : SYMTEN_PREC_F32);
        if (info) *info = p->info;
        if (out) *out = wrap(std::make_shared<Tensor>(*p->out_meta));
    });
}

int symten_contract(symten_t* out, symten_t A, symten_t B, int ncon, const int* legsA, const int* legsB,
                    const int* out_perm, int prec, void* stream) {
    return guard_on(stream, [&] {
        if (!out) fail(SYMTEN_E_INVAL, "null output");
        auto p = get_plan(T(A), T(B), ncon, legsA, legsB, out_perm, prec);
        *out = wrap(run_contraction(*p, T(A), T(B), S(stream)));
    });
}

int symten_contract_noalloc(symten_t out, symten_t A, symten_t B, int ncon, const int* legsA, const int* legsB,
                            const int* out_perm, int prec, void* stream) {
    return guard_on(stream, [&] {
        if (!out) fail(SYMTEN_E_INVAL, "contract_noalloc: null output tensor");
        auto p = cached_plan(T(A), T(B), ncon, legsA, legsB, out_perm, prec);
        contract_noalloc(T(out), T(A), T(B), p, S(stream));
    });
}

int symten_eigh(int count, const int* n, const double* const* A, const int* lda, double* const* w, const int* k,
                double* const* Z, void* stream) {
    return guard_on(stream, [&] {
        if (count < 0) fail(SYMTEN_E_INVAL, "eigh: negative count");
        if (count == 0) return;
        if (!n || !A || !lda || !w || !k || !Z) fail(SYMTEN_E_INVAL, "eigh: null array");
        std::vector<EighProblem> probs(count);
        for (int i = 0; i < count; ++i) {
            if (n[i] < 1 || lda[i] < n[i] || !A[i] || !w[i]) fail(SYMTEN_E_INVAL, "eigh: bad problem");
            if (k[i] < 0 || k[i] > n[i] || (k[i] > 0 && !Z[i])) fail(SYMTEN_E_INVAL, "eigh: bad vector count");
            if (!eigh_fits(n[i])) fail(SYMTEN_E_CAPACITY, "eigh: order above symten_eigh_max_order");
            probs[i].n = n[i];
            probs[i].lda = lda[i];
            probs[i].A = A[i];
            probs[i].w = w[i];
        }
        hipStream_t s = S(stream);
        auto wk = eigh_values(probs, s);
        eigh_status(*wk, s);   // synchronises s
        std::vector<std::vector<double>> wh(count);
        std::vector<const double*> whp(count);
        std::vector<int> kv(count);
        std::vector<double*> zs(count);
        for (int i = 0; i < count; ++i) {
            wh[i].resize(n[i]);
            HIPCHK(hipMemcpy(wh[i].data(), w[i], 8 * (size_t)n[i], hipMemcpyDeviceToHost));
            whp[i] = wh[i].data();
            kv[i] = k[i];
            zs[i] = Z[i];
        }
        eigh_vectors(*wk, kv, zs, whp, s);
    });
}

int symten_eigh_max_order(int* nmax) {
    return guard([&] {
        if (!nmax) fail(SYMTEN_E_INVAL, "null output");
        *nmax = eigh_max_order();
    });
}

int symten_match_blocks(symten_t A, symten_t B, int ncon, const int* legsA, const int* legsB, symten_pair* pairs,
                        int64_t pair_cap, int* out_labels, int64_t out_cap, int64_t* counts, void* stream) {
    return guard_on(stream, [&] {
        match_blocks(T(A), T(B), ncon, legsA, legsB, pairs, pair_cap, out_labels, out_cap, counts, S(stream));
    });
}

int symten_double_layer(symten_t* a_out, symten_t A, void* stream) {
    return guard_on(stream, [&] {
        if (!a_out) fail(SYMTEN_E_INVAL, "null output");
        *a_out = wrap(double_layer(T(A), S(stream)));
    });
}

int symten_enlarged_corner(symten_t* out, int which, symten_t C, symten_t Ta, symten_t Tb, symten_t a, int prec,
                           symten_plan_stats* info, void* stream) {
    return guard_on(stream, [&] {
        if (!out) fail(SYMTEN_E_INVAL, "null output");
        CornerResult r = corner(which, T(C), T(Ta), T(Tb), T(a), prec, S(stream));
        if (info) *info = r.info;
        *out = wrap(r.corner);
    });
}

int symten_enlarged_corner_single_layer(symten_t* out, int which, symten_t C, symten_t Ta, symten_t Tb, symten_t A,
                                        int prec, symten_plan_stats* info, void* stream) {
    return guard_on(stream, [&] {
        if (!out) fail(SYMTEN_E_INVAL, "null output");
        CornerResult r = corner_single_layer(which, T(C), T(Ta), T(Tb), T(A), prec, S(stream));
        if (info) *info = r.info;
        *out = wrap(r.corner);
    });
}

}  // extern "C"

// ---- batched corners ------------------------------------------------------
namespace {
struct BatchStep {
    std::vector<std::shared_ptr<ContractPlan>> plans;
    BufferPtr tasks, prefix, groups, ptrs, apanel, bpanel, out, ws;
    BufferPtr scatter;            // scatter tables when the GEMM writes the next step's A panels
    int ntasks = 0;
    int64_t npieces = 0;
    TileChoice tc;
    std::vector<GemmGroup> host_groups;
    std::vector<int64_t> c_base, a_base;
    std::vector<int> group_base;  // first group of each contraction
    int64_t ap = 0;               // elements of one plane of the A panels
    void* next_apanel = nullptr;  // the A panels the scatter epilogue writes
    std::vector<void*> table;     // host copy of the pointer table
    bool src_f64 = false, panel_f64 = false;
    Prec prec = Prec::F32;
    symten_plan_stats info{};
    int64_t copy_bytes = 0, gemm_bytes = 0;   // algorithmic bytes per launch
};
struct BatchState {
    int n = 0;
    BatchStep step[3];
    std::vector<TensorPtr> outs[3];
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> inputs;    // data pointers the tables were built for
    ~BatchState() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};
std::mutex g_batch_mu;
std::map<std::string, std::shared_ptr<BatchState>> g_batch;

// Concatenate the per-contraction plans of one step into one launch pair.
// fused_in: the previous step's GEMM writes this step's A panels (the A-side
// gathers are left out); fused_out: this step's GEMM writes the next step's A
// panels (no output buffer).
void build_step(BatchStep& B, const std::vector<const Tensor*>& As, const std::vector<const Tensor*>& Bs, int n,
                bool fused_in = false, bool fused_out = false) {
    std::vector<CopyTask> tasks;
    std::vector<GemmGroup> groups;
    std::vector<int64_t> a_base(n), b_base(n);
    int64_t ap = 0, bp = 0, cp = 0;
    B.c_base.assign(n, 0);
    B.group_base.assign(n, 0);
    B.info = {};
    for (int i = 0; i < n; ++i) {
        const ContractPlan& p = *B.plans[i];
        a_base[i] = ap;
        b_base[i] = bp;
        B.c_base[i] = cp;
        B.group_base[i] = (int)groups.size();
        ap += (p.a_panel_elems + 31) / 32 * 32;
        bp += (p.b_panel_elems + 31) / 32 * 32;
        cp += (p.out_elems + 31) / 32 * 32;
        add_info(B.info, p.info);
        size_t skipped = 0;
        for (CopyTask t : p.copies) {
            if (fused_in && t.src_buf == 0) {   // written by the previous step's GEMM
                ++skipped;
                continue;
            }
            if (t.src_buf == 0) t.src_buf = i;
            else if (t.src_buf == 1) t.src_buf = n + i;
            if (t.dst_buf == 2) { t.dst_buf = 2 * n; t.dst_off += a_base[i]; }
            else { t.dst_buf = 2 * n + 1; t.dst_off += b_base[i]; }
            tasks.push_back(t);
        }
        if (fused_in && skipped != p.a_maps.size())
            fail(SYMTEN_E_INVAL, "internal: fused step without a block map for every A-side gather");
        for (auto& g : p.groups) {
            GemmGroup x{};
            x.a_off = g.a_off + a_base[i];
            x.b_off = g.b_off + b_base[i];
            x.c_off = g.c_off + B.c_base[i];
            x.M = g.M;
            x.N = g.N;
            x.K = g.K;
            x.lda = x.ldb = g.lda;
            x.ldc = g.N;
            x.a_buf = 2 * n;
            x.b_buf = 2 * n + 1;
            x.c_buf = 2 * n + 2;
            groups.push_back(x);
        }
    }
    B.prec = B.plans[0]->prec;
    B.panel_f64 = B.plans[0]->panel_f64;
    B.src_f64 = As[0]->dtype == SYMTEN_F64;
    for (int i = 0; i < n; ++i)
        if (B.plans[i]->prec != B.prec || (As[i]->dtype == SYMTEN_F64) != B.src_f64)
            fail(SYMTEN_E_INVAL, "batched corners: inputs differ in storage type");
    const int pl = panel_planes(B.prec);
    if (pl > 1) {   // the lower planes follow the concatenated hi planes
        for (auto& t : tasks) t.lo_off = t.dst_buf == 2 * n ? ap : bp;
        for (auto& g : groups) {
            g.a_lo = ap;
            g.b_lo = bp;
        }
    }
    {
        std::vector<int64_t> sizes(2 * n + 3);
        for (int i = 0; i < n; ++i) { sizes[i] = As[i]->elems; sizes[n + i] = Bs[i]->elems; }
        sizes[2 * n] = pl * ap;
        sizes[2 * n + 1] = pl * bp;
        sizes[2 * n + 2] = cp;
        validate_tasks(tasks, sizes, pl);
        validate_groups(groups, sizes, panel_vw(B.prec), pl);
    }
    const size_t pe = panel_esize(B.prec) * pl;
    const size_t oe = B.src_f64 ? 8 : 4;
    B.a_base = a_base;
    B.ap = ap;
    B.apanel = device_alloc(std::max<int64_t>(ap, 1) * pe);
    B.bpanel = device_alloc(std::max<int64_t>(bp, 1) * pe);
    B.out = device_alloc(std::max<int64_t>(fused_out ? 1 : cp, 1) * oe);
    std::vector<int64_t> prefix;
    copy_prefix(tasks, prefix);
    B.ntasks = (int)tasks.size();
    B.npieces = prefix.back();
    upload_sync(B.tasks, tasks.data(), tasks.size() * sizeof(CopyTask));
    upload_sync(B.prefix, prefix.data(), prefix.size() * sizeof(int64_t));
    B.host_groups = groups;
    upload_sync(B.groups, groups.data(), groups.size() * sizeof(GemmGroup));
    B.ptrs = device_alloc(sizeof(void*) * (2 * n + 5));
    B.copy_bytes = symten::copy_bytes(tasks, oe, pe);
    B.gemm_bytes = symten::gemm_bytes(groups, pe, oe);
}

// Step K's GEMM writes step K1's A panels: the products of every output
// block that step K1 gathers go, split into bf16 planes, to the panel
// positions of step K1's A-side block maps (the same values and rounding as
// the gather of a stored product).  Step K's groups get scatter tables:
// per row its row block and the multi-index over the A-side free legs, per
// column the same over the B-side free legs, per (row block, column block)
// the panel offset and leg strides (d0 < 0: a block step K1 does not read).
void fuse_steps(BatchStep& K, const std::vector<const Tensor*>& As, const std::vector<const Tensor*>& Bs,
                const BatchStep& K1, int n) {
    std::vector<int> tab;
    const int pl = panel_planes(K.prec);
    int64_t written = 0;
    for (int i = 0; i < n; ++i)
        written += append_scatter_tables(*K.plans[i], *As[i], *Bs[i], *K1.plans[i], K1.a_base[i],
                                         K.host_groups.data() + K.group_base[i], tab);
    for (GemmGroup& G : K.host_groups) {
        G.s_buf = 2 * n + 3;
        G.c_buf = 2 * n + 4;
        G.c_lo = K1.ap;
    }
    validate_scatter(K.host_groups, tab, pl * std::max<int64_t>(K1.ap, 1), pl);
    upload_sync(K.scatter, tab.data(), tab.size() * sizeof(int));
    upload_sync(K.groups, K.host_groups.data(), K.host_groups.size() * sizeof(GemmGroup));
    K.next_apanel = K1.apanel->ptr;
    // algorithmic bytes: panels read, products written once in all planes
    const size_t pe = panel_esize(K.prec) * pl;
    K.gemm_bytes = 0;
    for (const GemmGroup& g : K.host_groups) K.gemm_bytes += (int64_t)pe * ((int64_t)g.M * g.K + (int64_t)g.N * g.K);
    K.gemm_bytes += (int64_t)pe * written;
}

void set_table(BatchStep& B, const std::vector<void*>& a, const std::vector<void*>& b) {
    const int n = (int)a.size();
    std::vector<void*> t(2 * n + 5, nullptr);
    for (int i = 0; i < n; ++i) { t[i] = a[i]; t[n + i] = b[i]; }
    t[2 * n] = B.apanel->ptr;
    t[2 * n + 1] = B.bpanel->ptr;
    t[2 * n + 2] = B.out->ptr;
    if (B.scatter) {
        t[2 * n + 3] = B.scatter->ptr;
        t[2 * n + 4] = B.next_apanel;
    }
    if (t != B.table) {
        HIPCHK(hipMemcpy(B.ptrs->ptr, t.data(), t.size() * sizeof(void*), hipMemcpyHostToDevice));
        B.table = t;
    }
}

// One step of a batch: gather launch, then grouped GEMM.  With tune = true
// (never under graph capture) the tile configuration is chosen first.
void run_step(BatchStep& B, hipStream_t s, bool tune = false) {
    profile_launch(copy_kernel_name(B.src_f64, B.prec) + ",batched", 0, 0, B.copy_bytes, s, [&] {
        copy_launch_dev((const CopyTask*)B.tasks->ptr, (const int64_t*)B.prefix->ptr, B.ntasks, B.npieces,
                        (void* const*)B.ptrs->ptr, B.src_f64, panel_dst_kind(B.prec), s);
    });
    auto launch = [&](int cfg) {
        // the split-K workspace lives with the step (a captured graph keeps
        // its address); it only grows while the shapes are being tuned
        if (B.tc.ws_bytes[cfg] > (B.ws ? (int64_t)B.ws->bytes : 0)) {
            if (!tune) fail(SYMTEN_E_INVAL, "internal: batched split-K workspace not sized before capture");
            B.ws = device_alloc(B.tc.ws_bytes[cfg]);
        }
        gemm_launch_dev((const TileWork*)B.tc.tiles[cfg]->ptr, B.tc.ntiles[cfg], (const GemmGroup*)B.groups->ptr,
                        (void* const*)B.ptrs->ptr, B.prec, cfg, s, B.tc.split(cfg, B.ws ? B.ws->ptr : nullptr),
                        B.scatter != nullptr);
    };
    if (tune) autotune_gemm(B.tc, B.host_groups, B.prec, launch, s);
    if (B.tc.cfg < 0) fail(SYMTEN_E_INVAL, "internal: batched GEMM launched before tuning");
    const int cfg = B.tc.cfg;
    profile_launch(gemm_kernel_name(B.prec, cfg, B.scatter != nullptr) + ",batched", B.info.useful_flops, B.info.gemm_flops, B.gemm_bytes,
                   s, [&] { launch(cfg); });
}

// The n outputs of a step as views into one buffer laid out like B.out.
std::vector<TensorPtr> step_outputs(const BatchStep& B, int n, const BufferPtr& buf) {
    std::vector<TensorPtr> outs(n);
    for (int i = 0; i < n; ++i) {
        auto t = std::make_shared<Tensor>(*B.plans[i]->out_meta);
        for (auto& b : t->blocks) b.offset += B.c_base[i];
        t->elems = B.c_base[i] + B.plans[i]->out_elems;
        t->buf = buf;
        t->meta_only = false;
        outs[i] = t;
    }
    return outs;
}
}  // namespace

extern "C" {

int symten_enlarged_corners_batched(int n, symten_t* out, const symten_t* Cs, const symten_t* Tas,
                                    const symten_t* Tbs, const symten_t* as, int prec, int use_graph,
                                    symten_plan_stats* info, void* stream) {
    return guard_on(stream, [&] {
        if (n <= 0 || !out || !Cs || !Tas || !Tbs || !as) fail(SYMTEN_E_INVAL, "batched corners: bad arguments");
        const hipStream_t s = S(stream);
        std::string key = std::to_string(n) + "|" + std::to_string(prec) + "|";
        std::vector<void*> inputs;
        for (int i = 0; i < n; ++i) {
            for (symten_t h : {Cs[i], Tas[i], Tbs[i], as[i]}) {
                check_device_tensor(T(h), "batched corners");
                if (!abelian(T(h).group)) fail(SYMTEN_E_UNSUPPORTED, "batched corners: U(1) or Z2 tensors only");
                key += tensor_signature(T(h)) + "&";
                inputs.push_back(T(h).data());
            }
        }
        std::shared_ptr<BatchState> st;
        {
            std::lock_guard<std::mutex> lk(g_batch_mu);
            auto it = g_batch.find(key);
            if (it != g_batch.end()) st = it->second;
        }
        // The chain of corner 1 with step 1's output ordered [xa, x1, u]:
        // step 2's products [x1, u, y, l] then reach step 3's A panels
        // (contracted over (l, u), u fastest) with consecutive rows on
        // consecutive positions.  Same corners as corner(1, ...).
        const std::vector<int> l1a{1}, l1b{0}, perm1{0, 2, 1}, l2a{0}, l2b{2}, l3a{3, 1}, l3b{0, 1};
        if (!st) {
            st = std::make_shared<BatchState>();
            st->n = n;
            std::vector<const Tensor*> A1, B1, B2, B3;
            for (int i = 0; i < n; ++i) {
                A1.push_back(&T(Cs[i]));
                B1.push_back(&T(Tas[i]));
                B2.push_back(&T(Tbs[i]));
                B3.push_back(&T(as[i]));
            }
            for (int i = 0; i < n; ++i)
                st->step[0].plans.push_back(get_plan(*A1[i], *B1[i], 1, l1a.data(), l1b.data(), perm1.data(), prec));
            build_step(st->step[0], A1, B1, n);
            st->outs[0] = step_outputs(st->step[0], n, st->step[0].out);
            std::vector<const Tensor*> A2;
            for (int i = 0; i < n; ++i) {
                A2.push_back(st->outs[0][i].get());
                st->step[1].plans.push_back(get_plan(*A2[i], *B2[i], 1, l2a.data(), l2b.data(), nullptr, prec));
            }
            // bf16 precisions: step 2's GEMM writes step 3's A panels itself
            const Prec p2 = st->step[1].plans[0]->prec;
            const bool fuse = p2 == Prec::BF16 || p2 == Prec::BF16X3 || p2 == Prec::BF16X6;
            build_step(st->step[1], A2, B2, n, false, fuse);
            st->outs[1] = step_outputs(st->step[1], n, st->step[1].out);
            std::vector<const Tensor*> A3;
            for (int i = 0; i < n; ++i) {
                A3.push_back(st->outs[1][i].get());
                st->step[2].plans.push_back(get_plan(*A3[i], *B3[i], 2, l3a.data(), l3b.data(), nullptr, prec));
            }
            build_step(st->step[2], A3, B3, n, fuse, false);
            if (fuse) fuse_steps(st->step[1], A2, B2, st->step[2], n);
            std::lock_guard<std::mutex> lk(g_batch_mu);
            if (g_batch.size() > 16) g_batch.clear();
            g_batch[key] = st;
        }
        if (st->inputs != inputs) {
            // (re)point the tables at the current input buffers; earlier calls
            // on any stream may still read them, so the device is drained first
            HIPCHK(hipDeviceSynchronize());
            std::vector<void*> c(n), t1(n), t4(n), a(n), o1(n), o2(n);
            const size_t es = st->step[0].src_f64 ? 8 : 4;
            for (int i = 0; i < n; ++i) {
                c[i] = inputs[4 * i];
                t1[i] = inputs[4 * i + 1];
                t4[i] = inputs[4 * i + 2];
                a[i] = inputs[4 * i + 3];
                o1[i] = (char*)st->step[0].out->ptr;
                o2[i] = (char*)st->step[1].out->ptr;
                (void)es;
            }
            set_table(st->step[0], c, t1);
            set_table(st->step[1], o1, t4);
            set_table(st->step[2], o2, a);
            st->inputs = inputs;
            if (st->exec) {
                (void)hipGraphExecDestroy(st->exec);
                (void)hipGraphDestroy(st->graph);
                st->exec = nullptr;
                st->graph = nullptr;
            }
        }
        // every call writes its corners into a buffer of its own (earlier
        // results stay valid): the last step's output entry of the pointer
        // table is set on s before the launches that read it
        BatchStep& last = st->step[2];
        BufferPtr result = device_alloc(std::max<int64_t>(last.out->bytes, 1));
        launch_set_pointer((void**)last.ptrs->ptr, 2 * n + 2, result->ptr, s);
        last.table[2 * n + 2] = result->ptr;
        bool tuned = true;
        for (int k = 0; k < 3; ++k) tuned = tuned && st->step[k].tc.cfg >= 0;
        if (!tuned) {
            // first use: an eager pass that also picks every step's tile shape
            for (int k = 0; k < 3; ++k) run_step(st->step[k], s, true);
        }
        if (use_graph) {
            if (!st->exec) {
                // Capture on a library stream (the caller's may be the null
                // stream, which cannot capture); nothing runs during capture.
                static hipStream_t cap = nullptr;
                if (!cap) HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
                HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
                try {
                    for (int k = 0; k < 3; ++k) run_step(st->step[k], cap);
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(cap, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                HIPCHK(hipStreamEndCapture(cap, &st->graph));
                HIPCHK(hipGraphInstantiate(&st->exec, st->graph, nullptr, nullptr, 0));
            }
            HIPCHK(hipGraphLaunch(st->exec, s));
        } else {
            for (int k = 0; k < 3; ++k) run_step(st->step[k], s);
        }
        if (info) {
            *info = {};
            for (int k = 0; k < 3; ++k) add_info(*info, st->step[k].info);
        }
        std::vector<TensorPtr> res = step_outputs(last, n, result);
        for (int i = 0; i < n; ++i) out[i] = wrap(res[i]);
    });
}

int ctm_env_create(ctm_env_t* env, const symten_t C[4], const symten_t Tt[4]) {
    return guard([&] {
        if (!env || !C || !Tt) fail(SYMTEN_E_INVAL, "null argument");
        auto* e = new ctm_env();
        try {
            for (int i = 0; i < 4; ++i) {
                e->C[i] = T(C[i]).buf ? C[i]->t : nullptr;
                e->T[i] = T(Tt[i]).buf ? Tt[i]->t : nullptr;
                if (!e->C[i] || !e->T[i]) fail(SYMTEN_E_INVAL, "environment tensors need device storage");
                if (e->C[i]->rank() != 2 || e->T[i]->rank() != 3) fail(SYMTEN_E_INVAL, "C must be rank 2 and T rank 3");
                if (e->C[i]->group != e->C[0]->group || e->T[i]->group != e->C[0]->group)
                    fail(SYMTEN_E_SYM, "environment: tensors of different symmetry groups");
            }
            rb_check(rocblas_create_handle(&e->rb), "rocblas_create_handle");
            HIPCHK(hipEventCreateWithFlags(&e->ev_start, hipEventDisableTiming));
            for (int i = 0; i < ctm_env::kAux; ++i) {
                HIPCHK(hipStreamCreateWithFlags(&e->aux[i], hipStreamNonBlocking));
                HIPCHK(hipEventCreateWithFlags(&e->ev_done[i], hipEventDisableTiming));
                rb_check(rocblas_create_handle(&e->rb_aux[i]), "rocblas_create_handle");
                rb_check(rocblas_set_stream(e->rb_aux[i], e->aux[i]), "rocblas_set_stream");
            }
        } catch (...) {
            delete e;
            throw;
        }
        *env = e;
    });
}

void ctm_env_destroy(ctm_env_t env) { delete env; }

int ctm_env_set(ctm_env_t env, int k, symten_t t) {
    return guard([&] {
        if (!env || k < 0 || k > 7) fail(SYMTEN_E_INVAL, "bad argument");
        Tensor& x = T(t);
        check_device_tensor(x, "ctm_env_set");
        if (x.rank() != (k < 4 ? 2 : 3)) fail(SYMTEN_E_INVAL, "C must be rank 2 and T rank 3");
        (k < 4 ? env->C[k] : env->T[k - 4]) = t->t;
    });
}

int symten_profile_begin(void) {
    return guard([&] { profile_begin(); });
}

int symten_profile_end(symten_kernel_stat* out, int cap, int* n) {
    return guard([&] {
        if (!n) fail(SYMTEN_E_INVAL, "null count");
        std::vector<symten_kernel_stat> v = profile_end();
        *n = (int)v.size();
        if (out)
            for (int i = 0; i < std::min(cap, *n); ++i) out[i] = v[i];
    });
}

int ctm_env_get(ctm_env_t env, int k, symten_t* t) {
    return guard([&] {
        if (!env || !t || k < 0 || k > 7) fail(SYMTEN_E_INVAL, "bad argument");
        *t = wrap(k < 4 ? env->C[k] : env->T[k - 4]);
    });
}

int ctm_move_singular_values(ctm_env_t env, double* s, int64_t cap, int64_t* n) {
    return guard([&] {
        if (!env || !n) fail(SYMTEN_E_INVAL, "bad argument");
        *n = (int64_t)env->svals.size();
        if (s) std::copy(env->svals.begin(), env->svals.begin() + std::min<int64_t>(cap, *n), s);
    });
}

int ctm_move_projectors(ctm_env_t env, symten_t* P, symten_t* Pt) {
    return guard([&] {
        if (!env || !env->P.t) fail(SYMTEN_E_INVAL, "no move has run");
        if (P) *P = wrap(env->P.t);
        if (Pt) *Pt = wrap(env->Pt.t);
    });
}

int ctm_move(ctm_env_t env, symten_t a_h, int dir, int chi, int prec, ctm_move_stats* st, void* stream) {
    const int rc = guard_on(stream, [&] {
        if (!env) fail(SYMTEN_E_INVAL, "null environment");
        if (dir < CTM_LEFT || dir > CTM_BOTTOM) fail(SYMTEN_E_INVAL, "ctm_move: direction must be 0..3");
        if (chi < 1) fail(SYMTEN_E_INVAL, "chi must be positive");
        Tensor& a = T(a_h);
        check_device_tensor(a, "ctm_move(a)");
        if (a.rank() != 4) fail(SYMTEN_E_INVAL, "a must have rank 4");
        const hipStream_t s = S(stream);
        const bool f64 = prec == SYMTEN_PREC_F64;
        env->degen_tol = ctm_env::degenerate_tol(prec);
        for (int i = 0; i < 4; ++i) {
            if ((env->C[i]->dtype == SYMTEN_F64) != f64 || (env->T[i]->dtype == SYMTEN_F64) != f64 ||
                (a.dtype == SYMTEN_F64) != f64)
                fail(SYMTEN_E_INVAL, "ctm_move: storage types do not match the precision");
            if (env->C[i]->group != a.group || env->T[i]->group != a.group)
                fail(SYMTEN_E_SYM, "ctm_move: environment and site tensor have different symmetry groups");
        }
        if (a.group == SYMTEN_SU2) {
            if (dir == CTM_LEFT) {
                move_su2(env, a, chi, prec, st, s);
                return;
            }
            // the network turned as in the U(1) case; the reversed legs go
            // through the S^z basis (su2_permute_flip).  Over four turns every
            // T's D^2 leg is reversed twice, which multiplies its half-integer
            // spins by -1: undone at the end so that the environment matches
            // the caller's a again.
            auto turn = [&](std::array<TensorPtr, 4>& C, std::array<TensorPtr, 4>& Tt, TensorPtr& ar) {
                const std::array<TensorPtr, 4> Cn{C[1], C[2], C[3], C[0]};
                const std::array<TensorPtr, 4> Tn{su2_permute_flip(*Tt[1], {0, 1, 2}, {1}, s), Tt[2],
                                                  su2_permute_flip(*Tt[3], {0, 1, 2}, {1}, s), Tt[0]};
                ar = su2_permute_flip(*ar, {1, 2, 3, 0}, {1, 3}, s);
                C = Cn;
                Tt = Tn;
            };
            std::array<TensorPtr, 4> C{env->C[0], env->C[1], env->C[2], env->C[3]};
            std::array<TensorPtr, 4> Tt{env->T[0], env->T[1], env->T[2], env->T[3]};
            const std::array<TensorPtr, 4> C0 = C, T0 = Tt;
            TensorPtr ar = a_h->t;
            for (int r = 0; r < dir; ++r) turn(C, Tt, ar);
            for (int i = 0; i < 4; ++i) { env->C[i] = C[i]; env->T[i] = Tt[i]; }
            try {
                move_su2(env, *ar, chi, prec, st, s);
            } catch (...) {
                for (int i = 0; i < 4; ++i) { env->C[i] = C0[i]; env->T[i] = T0[i]; }
                throw;
            }
            for (int i = 0; i < 4; ++i) { C[i] = env->C[i]; Tt[i] = env->T[i]; }
            for (int r = dir; r < 4; ++r) turn(C, Tt, ar);
            for (int i = 0; i < 4; ++i) {
                env->C[i] = C[i];
                env->T[i] = su2_sign_half_integer(*Tt[i], 1, s);
            }
            return;
        }
        if (dir == CTM_LEFT) {
            move_u1_left(env, a, chi, prec, st, s);
            return;
        }
        // the other directions: the left move of the network turned by `dir`
        // quarter turns counterclockwise, then turned back
        std::array<TensorPtr, 4> C{env->C[0], env->C[1], env->C[2], env->C[3]};
        std::array<TensorPtr, 4> Tt{env->T[0], env->T[1], env->T[2], env->T[3]};
        TensorPtr ar = a_h->t;
        for (int r = 0; r < dir; ++r) rotate_ccw(C, Tt, ar);
        for (int i = 0; i < 4; ++i) { env->C[i] = C[i]; env->T[i] = Tt[i]; }
        try {
            move_u1_left(env, *ar, chi, prec, st, s);
        } catch (...) {
            for (int r = dir; r < 4; ++r) rotate_ccw(C, Tt, ar);
            for (int i = 0; i < 4; ++i) { env->C[i] = C[i]; env->T[i] = Tt[i]; }
            throw;
        }
        for (int i = 0; i < 4; ++i) { C[i] = env->C[i]; Tt[i] = env->T[i]; }
        for (int r = dir; r < 4; ++r) rotate_ccw(C, Tt, ar);
        for (int i = 0; i < 4; ++i) { env->C[i] = C[i]; env->T[i] = Tt[i]; }
    });
    // The move ends with its stream synchronised.  Its read-back of the
    // spectrum already waits for the stream once; returning while the last
    // kernels (vectors, projectors, renormalisation) still ran let the
    // caller enqueue the next move behind them, and back-to-back D = 6,
    // chi = 64 moves then took 8.5-8.6 ms against 6.9 ms with this wait
    // (measured with host timers; the difference does not appear under a
    // kernel trace, which gives every dispatch its own completion signal).
    if (rc != SYMTEN_OK) return rc;
    return guard_on(stream, [&] { HIPCHK(hipStreamSynchronize(S(stream))); });
}

int ctm_cell_create(ctm_env_t* env, int Lx, int Ly, const symten_t* C, const symten_t* Tt) {
    return guard([&] {
        if (!env || !C || !Tt || Lx < 1 || Ly < 1 || Lx > 16 || Ly > 16) fail(SYMTEN_E_INVAL, "bad argument");
        // the handles and side streams of a 1x1 environment on site (0, 0)
        ctm_env_t e = nullptr;
        const int rc = ctm_env_create(&e, C, Tt);
        if (rc != SYMTEN_OK) fail(rc, g_err);
        e->Lx = Lx;
        e->Ly = Ly;
        for (int i = 0; i < 4 * Lx * Ly; ++i) {
            Tensor &c = T(C[i]), &t = T(Tt[i]);
            if (!c.buf || !t.buf || c.rank() != 2 || t.rank() != 3 || c.group != e->C[0]->group ||
                t.group != e->C[0]->group || !abelian(c.group)) {
                delete e;
                fail(SYMTEN_E_INVAL, "cell: C rank 2 and T rank 3 with device storage, one abelian group");
            }
            e->cC.push_back(C[i]->t);
            e->cT.push_back(Tt[i]->t);
        }
        *env = e;
    });
}

int ctm_cell_get(ctm_env_t env, int x, int y, int k, symten_t* t) {
    return guard([&] {
        if (!env || !t || env->Lx < 1) fail(SYMTEN_E_INVAL, "not a unit-cell environment");
        if (x < 0 || y < 0 || x >= env->Lx || y >= env->Ly || k < 0 || k > 7) fail(SYMTEN_E_INVAL, "bad index");
        const int i = 4 * (x * env->Ly + y) + (k & 3);
        *t = wrap(k < 4 ? env->cC[i] : env->cT[i]);
    });
}

int ctm_cell_move(ctm_env_t env, const symten_t* a_h, int dir, int chi, int prec, void* stream) {
    const int rc = guard_on(stream, [&] {
        if (!env || !a_h || env->Lx < 1) fail(SYMTEN_E_INVAL, "not a unit-cell environment");
        if (dir < CTM_LEFT || dir > CTM_BOTTOM) fail(SYMTEN_E_INVAL, "ctm_cell_move: direction must be 0..3");
        if (chi < 1) fail(SYMTEN_E_INVAL, "chi must be positive");
        const bool f64 = prec == SYMTEN_PREC_F64;
        env->degen_tol = ctm_env::degenerate_tol(prec);
        int Lx = env->Lx, Ly = env->Ly;
        std::vector<TensorPtr> a;
        for (int i = 0; i < Lx * Ly; ++i) {
            Tensor& t = T(a_h[i]);
            check_device_tensor(t, "ctm_cell_move(a)");
            if (t.rank() != 4 || t.group != env->cC[0]->group) fail(SYMTEN_E_INVAL, "cell: a is rank 4, the cell's group");
            if ((t.dtype == SYMTEN_F64) != f64) fail(SYMTEN_E_INVAL, "cell: storage types do not match the precision");
            a.push_back(a_h[i]->t);
        }
        for (auto& x : env->cC)
            if ((x->dtype == SYMTEN_F64) != f64) fail(SYMTEN_E_INVAL, "cell: storage types do not match the precision");
        // turn the cell `dir` quarter turns: site (x, y) -> (y, Lx - 1 - x),
        // every site's environment and tensor turned as in the 1x1 case
        auto turn = [&](int times) {
            for (int r = 0; r < times; ++r) {
                std::vector<TensorPtr> nC(4 * Lx * Ly), nT(4 * Lx * Ly), na(Lx * Ly);
                for (int x = 0; x < Lx; ++x)
                    for (int y = 0; y < Ly; ++y) {
                        std::array<TensorPtr, 4> Cs, Ts;
                        for (int i = 0; i < 4; ++i) {
                            Cs[i] = env->cC[4 * (x * Ly + y) + i];
                            Ts[i] = env->cT[4 * (x * Ly + y) + i];
                        }
                        TensorPtr ar = a[x * Ly + y];
                        rotate_ccw(Cs, Ts, ar);
                        const int nx = y, ny = Lx - 1 - x, nLy = Lx;
                        for (int i = 0; i < 4; ++i) {
                            nC[4 * (nx * nLy + ny) + i] = Cs[i];
                            nT[4 * (nx * nLy + ny) + i] = Ts[i];
                        }
                        na[nx * nLy + ny] = ar;
                    }
                std::swap(Lx, Ly);
                env->Lx = Lx;
                env->Ly = Ly;
                env->cC = nC;
                env->cT = nT;
                a = na;
            }
        };
        turn(dir);
        try {
            cell_left_move(env, a, chi, prec, S(stream));
        } catch (...) {
            turn((4 - dir) % 4);
            throw;
        }
        turn((4 - dir) % 4);
    });
    // ends with its stream synchronised, as ctm_move does (same reason)
    if (rc != SYMTEN_OK) return rc;
    return guard_on(stream, [&] { HIPCHK(hipStreamSynchronize(S(stream))); });
}

int ctm_cell_site_partition(ctm_env_t env, int x, int y, symten_t a, int block, double* kappa, double* z,
                            void* stream) {
    return guard_on(stream, [&] {
        if (!env || !kappa || env->Lx < 1) fail(SYMTEN_E_INVAL, "not a unit-cell environment");
        if (x < 0 || y < 0 || x >= env->Lx || y >= env->Ly) fail(SYMTEN_E_INVAL, "bad site");
        if (block != 1 && block != 2) fail(SYMTEN_E_INVAL, "block must be 1 or 2");
        Tensor& at = T(a);
        check_device_tensor(at, "ctm_cell_site_partition(a)");
        ctm_env site;                     // a view of site (x, y)'s environment
        for (int i = 0; i < 4; ++i) {
            site.C[i] = env->cC[4 * (x * env->Ly + y) + i];
            site.T[i] = env->cT[4 * (x * env->Ly + y) + i];
        }
        double zz[4];
        *kappa = site_partition(&site, a->t, block, zz, S(stream));
        if (z) std::copy(zz, zz + 4, z);
    });
}

int ctm_site_partition(ctm_env_t env, symten_t a, int block, double* kappa, double* z, void* stream) {
    return guard_on(stream, [&] {
        if (!env || !kappa) fail(SYMTEN_E_INVAL, "null argument");
        if (block != 1 && block != 2) fail(SYMTEN_E_INVAL, "block must be 1 or 2");
        Tensor& at = T(a);
        check_device_tensor(at, "ctm_site_partition(a)");
        if (env->C[0]->group != at.group || env->Lx > 0)
            fail(SYMTEN_E_INVAL, "ctm_site_partition: a 1x1 environment of a's symmetry group");
        if (at.rank() != 4) fail(SYMTEN_E_INVAL, "a must have rank 4");
        double zz[4];
        *kappa = site_partition(env, a->t, block, zz, S(stream));
        if (z) std::copy(zz, zz + 4, z);
    });
}

int ctm_expectation(ctm_env_t env, symten_t a, int n, int m, const symten_t* sites, double* value, void* stream) {
    return guard_on(stream, [&] {
        if (!env || !sites || !value) fail(SYMTEN_E_INVAL, "null argument");
        if (n < 1 || m < 1 || n > 2 || m > 2) fail(SYMTEN_E_INVAL, "ctm_expectation: patch of 1 or 2 columns and rows");
        Tensor& at = T(a);
        check_device_tensor(at, "ctm_expectation(a)");
        if (!abelian(at.group) || env->C[0]->group != at.group)
            fail(SYMTEN_E_UNSUPPORTED, "ctm_expectation: U(1) or Z2 tensors only");
        std::vector<TensorPtr> b;
        for (int k = 0; k < n * m; ++k) {
            Tensor& bt = T(sites[k]);
            check_device_tensor(bt, "ctm_expectation(site)");
            if (bt.group != at.group || bt.rank() != 4) fail(SYMTEN_E_INVAL, "ctm_expectation: sites are rank-4 tensors of a's group");
            for (int l = 0; l < 4; ++l)
                if (bt.legs[l].dir != at.legs[l].dir || bt.legs[l].q != at.legs[l].q || bt.legs[l].d != at.legs[l].d)
                    fail(SYMTEN_E_LEGS, "ctm_expectation: a site's legs differ from a's");
            b.push_back(sites[k]->t);
        }
        *value = expectation(env, a->t, n, m, b, S(stream));
    });
}

int ctm_heisenberg_bond_energy(ctm_env_t env, symten_t A, double* e_h, double* e_v, void* stream) {
    return guard_on(stream, [&] {
        if (!env || !e_h || !e_v) fail(SYMTEN_E_INVAL, "null argument");
        Tensor& At = T(A);
        check_device_tensor(At, "ctm_heisenberg_bond_energy(A)");
        if ((At.group != SYMTEN_U1 && At.group != SYMTEN_SU2 && At.group != SYMTEN_Z2) || At.rank() != 5 ||
            env->C[0]->group != At.group || env->Lx > 0)
            fail(SYMTEN_E_INVAL, "ctm_heisenberg_bond_energy: A is a rank-5 U(1), SU(2) or Z2 tensor of a 1x1 "
                                 "environment's group");
        hipStream_t s = S(stream);
        if (At.group == SYMTEN_Z2) {
            // spin 1/2 in the spin-flip parity basis |+-> = (|up> +- |down>)/sqrt2
            // (labels 0, 1): Sx = diag(1/2, -1/2) keeps the parity, Sz and
            // Sy = i J with J = [[0, 1/2], [-1/2, 0]] flip it, so
            // S_i . S_j = Sx Sx + Sz Sz - J J with real operators
            const Leg& p = At.legs[0];
            if (p.q != std::vector<int>{0, 1} || p.d != std::vector<int>{1, 1})
                fail(SYMTEN_E_INVAL, "ctm_heisenberg_bond_energy: the Z2 physical leg is {0: 1, 1: 1} (spin 1/2)");
            const double sx[4] = {0.5, 0.0, 0.0, -0.5}, sz[4] = {0.0, 0.5, 0.5, 0.0}, jy[4] = {0.0, 0.5, -0.5, 0.0};
            TensorPtr a = double_layer(At, s);
            TensorPtr bx = double_layer(At, s, sx), bz = double_layer(At, s, sz), bj = double_layer(At, s, jy);
            auto bond = [&](int n, int m) {
                return expectation(env, a, n, m, {bx, bx}, s) + expectation(env, a, n, m, {bz, bz}, s) -
                       expectation(env, a, n, m, {bj, bj}, s);
            };
            *e_h = bond(2, 1);
            *e_v = bond(1, 2);
            return;
        }
        const bool su2 = At.group == SYMTEN_SU2;
        if (su2 && (At.legs[0].q.size() != 1 || At.legs[0].d[0] != 1))
            fail(SYMTEN_E_INVAL, "ctm_heisenberg_bond_energy: the SU(2) physical leg is one multiplet");
        // physical states: charges 2m = -2S, -2S+2, ..., 2S, one state each
        // (for SU(2): the S^z states of the physical multiplet)
        Leg ph = At.legs[0];
        if (su2) {
            const int tS = ph.q[0];
            ph.q.clear();
            ph.d.clear();
            for (int tm = -tS; tm <= tS; tm += 2) { ph.q.push_back(tm); ph.d.push_back(1); }
        }
        const int np = ph.size();
        if (np < 2 || np > kMaxOpStates) fail(SYMTEN_E_INVAL, "ctm_heisenberg_bond_energy: spin 1/2 .. 7/2");
        for (int k = 0; k < np; ++k)
            if ((int)ph.q.size() != np || ph.d[k] != 1 || ph.q[k] != -(np - 1) + 2 * k)
                fail(SYMTEN_E_INVAL, "ctm_heisenberg_bond_energy: physical charges must be 2m, m = -S..S");
        const double S2 = 0.5 * (np - 1);
        std::vector<double> sz(np * np, 0.0), sp(np * np, 0.0), sm(np * np, 0.0);
        for (int k = 0; k < np; ++k) {
            const double mz = -S2 + k;
            sz[k * np + k] = mz;
            if (k + 1 < np) {
                const double c = std::sqrt(S2 * (S2 + 1.0) - mz * (mz + 1.0));
                sp[(k + 1) * np + k] = c;       // <m+1| S+ |m>
                sm[k * np + (k + 1)] = c;       // <m| S- |m+1>
            }
        }
        // SU(2): the spin operators are not invariant, so the state is
        // measured through its S^z components -- the environment expanded
        // (su2_to_u1) and the double layers built in the same S^z basis of
        // the fused multiplets -- on the U(1) path; the value is the same
        ctm_env expanded;
        ctm_env* e = env;
        TensorPtr a, bz, bp, bm;
        if (su2) {
            for (int i = 0; i < 4; ++i) {
                expanded.C[i] = su2_to_u1(*env->C[i], s);
                expanded.T[i] = su2_to_u1(*env->T[i], s);
            }
            e = &expanded;
            a = double_layer_su2_sz(At, nullptr, s);
            bz = double_layer_su2_sz(At, sz.data(), s);
            bp = double_layer_su2_sz(At, sp.data(), s);
            bm = double_layer_su2_sz(At, sm.data(), s);
        } else {
            a = double_layer(At, s);
            bz = double_layer(At, s, sz.data());
            bp = double_layer(At, s, sp.data());
            bm = double_layer(At, s, sm.data());
        }
        // S_i . S_j = Sz Sz + (S+ S- + S- S+) / 2 on the pair (left, right) or (top, bottom)
        auto bond = [&](int n, int m) {
            return expectation(e, a, n, m, {bz, bz}, s) +
                   0.5 * (expectation(e, a, n, m, {bp, bm}, s) + expectation(e, a, n, m, {bm, bp}, s));
        };
        *e_h = bond(2, 1);
        *e_v = bond(1, 2);
    });
}

int symten_double_layer_op(symten_t* b_out, symten_t A, const double* op, void* stream) {
    return guard_on(stream, [&] {
        if (!b_out || !op) fail(SYMTEN_E_INVAL, "null argument");
        *b_out = wrap(double_layer(T(A), S(stream), op));
    });
}

int ctm_run(ctm_env_t env, symten_t a, const ctm_run_opts* o, ctm_run_result* r, void* stream) {
    return guard_on(stream, [&] {
        if (!env || !o || !r) fail(SYMTEN_E_INVAL, "null argument");
        if (o->chi < 1 || o->max_steps < 1 || (o->block != 1 && o->block != 2) || !(o->tol >= 0.0))
            fail(SYMTEN_E_INVAL, "ctm_run: bad options");
        Tensor& at = T(a);
        check_device_tensor(at, "ctm_run(a)");
        if (env->C[0]->group != at.group || env->Lx > 0)
            fail(SYMTEN_E_INVAL, "ctm_run: a 1x1 environment of a's symmetry group");
        ctm_run_result res{};
        double z[4], prev_level = 0.0;
        for (int chi = o->chi;; chi *= 2) {
            // steps at fixed chi until the value moves by less than tol, or max_steps
            double v = site_partition(env, a->t, o->block, z, S(stream));
            double d1 = 0.0, d2 = 0.0;          // the last two changes
            int st = 0;
            while (st < o->max_steps) {
                for (int dir = CTM_LEFT; dir <= CTM_BOTTOM; ++dir) {
                    const int rc = ctm_move(env, a, dir, chi, o->prec, nullptr, stream);
                    if (rc != SYMTEN_OK) fail(rc, g_err);
                }
                ++st;
                const double nv = site_partition(env, a->t, o->block, z, S(stream));
                d2 = d1;
                d1 = std::fabs(nv - v);
                v = nv;
                if (d1 < o->tol) break;
            }
            res.err_steps = std::max(d1, d2);
            res.steps = st;
            res.total_steps += st;
            res.err_chi = res.levels > 0 ? std::fabs(v - prev_level) : 0.0;
            res.kappa = v;
            res.chi = chi;
            ++res.levels;
            if ((res.levels > 1 && res.err_chi < o->tol) || 2 * (int64_t)chi > o->chi_max) break;
            prev_level = v;
        }
        res.error = std::max(res.err_steps, res.err_chi);
        *r = res;
    });
}

}  // extern "C"
