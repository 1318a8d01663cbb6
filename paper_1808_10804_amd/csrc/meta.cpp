// Host bookkeeping of libsymten: allowed-block enumeration, contraction
// planning (charge-sector grouping of matched block pairs), plan execution,
// the double layer, and a caching device allocator.
#include <charconv>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <numeric>
#include <set>
#include <sstream>

#include "internal.hpp"

namespace symten {


// gather destination kind for the panels of a precision (see copy_kernel)
int panel_dst_kind(Prec p) {
    switch (p) {
        case Prec::F64: return 1;
        case Prec::F32: return 0;
        case Prec::BF16: return 2;
        case Prec::BF16X3: return 3;
        default: return 5;
    }
}

std::string copy_kernel_name(bool src64, Prec p) {
    static const char* dst[] = {"f64", "f32", "bf16", "bf16x2", "bf16x3"};
    return std::string("copy_kernel<") + (src64 ? "f64" : "f32") + "," + dst[(int)p] + ">";
}

// ------------------------------------------------------------------ errors
[[noreturn]] void fail(int code, const std::string& msg) { throw Error(code, msg); }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        std::ostringstream os;
        os << what << ": " << hipGetErrorString(e);
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) throw Error(SYMTEN_E_NOMEM, os.str());
        throw Error(SYMTEN_E_HIP, os.str());
    }
}

// ------------------------------------------------------------- device pool
namespace {
thread_local hipStream_t tl_stream = nullptr;
thread_local bool tl_stream_set = false;
}  // namespace

StreamScope::StreamScope(hipStream_t s) : prev(tl_stream), prev_set(tl_stream_set) {
    tl_stream = s;
    tl_stream_set = true;
}
StreamScope::~StreamScope() {
    tl_stream = prev;
    tl_stream_set = prev_set;
}
bool call_stream_set() { return tl_stream_set; }
hipStream_t call_stream() { return tl_stream; }

namespace {
struct FreeBlock {
    void* ptr;
    hipStream_t stream;   // stream that released it
    hipEvent_t ev;        // recorded on `stream` at release (null: already idle)
};
struct Pool {
    std::mutex mu;
    std::multimap<size_t, FreeBlock> free_;   // capacity -> block
    std::vector<hipEvent_t> idle_events;
    size_t held = 0;
    hipEvent_t take_event() {   // under mu
        if (!idle_events.empty()) {
            hipEvent_t e = idle_events.back();
            idle_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }
};
Pool& pool() {
    static Pool* p = new Pool();   // leaked on purpose: buffers may outlive statics
    return *p;
}
size_t round_cap(size_t b) {
    if (b < 4096) return 4096;
    // round up to a multiple of 1/8 of the next power of two
    size_t p = 1;
    while (p < b) p <<= 1;
    size_t step = std::max<size_t>(p / 8, 4096);
    return (b + step - 1) / step * step;
}
}  // namespace

namespace {
struct UserAllocator {
    std::mutex mu;
    void* (*alloc)(size_t, void*) = nullptr;
    void (*free_fn)(void*, size_t, void*) = nullptr;
    void* ctx = nullptr;
    uint64_t gen = 0;  // bumped by every registration
};
UserAllocator& user_allocator() {
    static UserAllocator* u = new UserAllocator();
    return *u;
}
}  // namespace

void set_user_allocator(void* (*alloc)(size_t, void*), void (*free_fn)(void*, size_t, void*), void* ctx) {
    UserAllocator& u = user_allocator();
    std::lock_guard<std::mutex> lk(u.mu);
    u.alloc = alloc;
    u.free_fn = free_fn;
    u.ctx = ctx;
    ++u.gen;
}

BufferPtr device_alloc(size_t bytes) {
    auto b = std::make_shared<DeviceBuffer>();
    b->bytes = bytes;
    if (bytes == 0) return b;
    const size_t cap = round_cap(bytes);
    {
        // the registration is copied under the lock and the allocator called
        // outside it: the allocator may free library buffers (a garbage
        // collector running in it), whose release takes the same lock
        UserAllocator& u = user_allocator();
        std::unique_lock<std::mutex> lk(u.mu);
        void* (*alloc)(size_t, void*) = u.alloc;
        void (*free_fn)(void*, size_t, void*) = u.free_fn;
        void* ctx = u.ctx;
        const uint64_t gen = u.gen;
        lk.unlock();
        if (alloc) {
            b->ptr = alloc(cap, ctx);
            if (!b->ptr) fail(SYMTEN_E_NOMEM, "registered allocator returned null for " + std::to_string(cap) + " bytes");
            b->cap = cap;
            b->user_free = free_fn;
            b->user_ctx = ctx;
            b->user_gen = gen;
            return b;
        }
    }
    const hipStream_t cur = call_stream();
    b->stream = cur;
    {
        Pool& P = pool();
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.free_.lower_bound(cap);
        if (it != P.free_.end() && it->first <= cap * 2) {
            const FreeBlock fb = it->second;
            if (fb.ev) {
                // the block's last users were queued on fb.stream: a call on
                // another stream waits for them (same stream: queue order)
                if (fb.stream != cur) HIPCHK(hipStreamWaitEvent(cur, fb.ev, 0));
                P.idle_events.push_back(fb.ev);
            }
            b->ptr = fb.ptr;
            b->cap = it->first;
            P.free_.erase(it);
            P.held -= b->cap;
            return b;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cap);
    if (e != hipSuccess) {
        // release cached blocks and retry once
        (void)hipGetLastError();
        Pool& P = pool();
        {
            std::lock_guard<std::mutex> lk(P.mu);
            (void)hipDeviceSynchronize();
            for (auto& kv : P.free_) {
                (void)hipFree(kv.second.ptr);
                if (kv.second.ev) P.idle_events.push_back(kv.second.ev);
            }
            P.free_.clear();
            P.held = 0;
        }
        e = hipMalloc(&p, cap);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(SYMTEN_E_NOMEM, "device allocation of " + std::to_string(cap) + " bytes failed");
        }
    }
    b->ptr = p;
    b->cap = cap;
    return b;
}

DeviceBuffer::~DeviceBuffer() {
    if (!ptr) return;
    if (user_free) {
        // A buffer outliving its allocator's registration is not handed back:
        // the caller may have torn that allocator down (interpreter exit).
        UserAllocator& u = user_allocator();
        std::unique_lock<std::mutex> lk(u.mu);
        const bool current = u.gen == user_gen;
        lk.unlock();
        if (current) user_free(ptr, cap, user_ctx);
        return;
    }
    const hipStream_t rs = call_stream_set() ? call_stream() : stream;
    Pool& P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    hipEvent_t ev = P.take_event();
    if (ev && hipEventRecord(ev, rs) != hipSuccess) {
        // no event on that stream (e.g. it no longer exists): wait for the
        // device instead, after which the block is idle
        (void)hipGetLastError();
        (void)hipDeviceSynchronize();
        P.idle_events.push_back(ev);
        ev = nullptr;
    } else if (!ev) {
        (void)hipDeviceSynchronize();
    }
    P.free_.emplace(cap, FreeBlock{ptr, rs, ev});
    P.held += cap;
}

// ------------------------------------------------------------------ tensors
void Tensor::rebuild_index() {
    memo.reset();
    index.clear();
    for (size_t i = 0; i < blocks.size(); ++i) {
        std::vector<int> key = blocks[i].q;
        if (!blocks[i].tree.empty()) {
            key.push_back(-1);   // spins are >= 0: the marker cannot collide
            key.insert(key.end(), blocks[i].tree.begin(), blocks[i].tree.end());
        }
        index[key] = (int)i;
    }
}

int64_t enumerate_blocks(Tensor& t) {
    const int R = t.rank();
    t.blocks.clear();
    std::vector<int> sidx(R, 0);
    int64_t off = 0;
    if (R == 0) return 0;
    for (const auto& l : t.legs)
        if (l.q.empty()) { t.rebuild_index(); return 0; }
    while (true) {
        long s = 0;
        for (int l = 0; l < R; ++l) s += (long)t.legs[l].dir * t.legs[l].q[sidx[l]];
        if (cnorm(s - t.flux, charge_mod(t.group)) == 0) {
            Block b;
            b.q.resize(R);
            b.shape.resize(R);
            b.stride.resize(R);
            int64_t sz = 1;
            for (int l = 0; l < R; ++l) {
                b.q[l] = t.legs[l].q[sidx[l]];
                b.shape[l] = t.legs[l].d[sidx[l]];
                sz *= b.shape[l];
            }
            int64_t st = 1;
            for (int l = R - 1; l >= 0; --l) { b.stride[l] = st; st *= b.shape[l]; }
            b.offset = off;
            b.size = sz;
            off += sz;
            t.blocks.push_back(std::move(b));
        }
        int l = R - 1;
        while (l >= 0 && ++sidx[l] == (int)t.legs[l].q.size()) { sidx[l] = 0; --l; }
        if (l < 0) break;
    }
    t.rebuild_index();
    return off;
}

std::string tensor_signature(const Tensor& t) {
    {
        std::lock_guard<std::mutex> lk(t.memo.mu);
        if (t.memo.valid) return t.memo.sig;
    }
    // the same fields as before, appended with std::to_chars (a stream was
    // the host cost of planning a move's new tensors)
    std::string sig;
    sig.reserve(32 + 16 * t.legs.size() + 48 * t.blocks.size());
    char buf[24];
    auto put = [&](int64_t v, char sep) {
        const auto r = std::to_chars(buf, buf + sizeof(buf), v);
        sig.append(buf, r.ptr);
        if (sep) sig.push_back(sep);
    };
    sig.push_back('g');
    put(t.group, 'f');
    put(t.flux, 't');
    put(t.dtype, '|');
    for (auto& l : t.legs) {
        put(l.dir, ':');
        for (size_t i = 0; i < l.q.size(); ++i) {
            put(l.q[i], 'x');
            put(l.d[i], ',');
        }
        sig.push_back(';');
    }
    sig.push_back('|');
    for (auto& b : t.blocks) {
        for (int x : b.q) put(x, ',');
        for (int x : b.tree) {
            sig.push_back('t');
            put(x, 0);
        }
        sig.push_back('@');
        put(b.offset, '/');
        for (auto st : b.stride) put(st, ',');
        sig.push_back(';');
    }
    std::lock_guard<std::mutex> lk(t.memo.mu);
    t.memo.sig = std::move(sig);
    t.memo.valid = true;
    return t.memo.sig;
}

void check_device_tensor(const Tensor& t, const char* what) {
    if (t.meta_only) fail(SYMTEN_E_INVAL, std::string(what) + ": tensor has no device storage");
}

// ------------------------------------------------------------- copy tasks
static void simplify_task(CopyTask& t) {
    // drop unit dims, merge dims contiguous in both source and destination
    int n = 0;
    int dims[kMaxCopyRank];
    int64_t ss[kMaxCopyRank], ds[kMaxCopyRank];
    for (int k = 0; k < t.rank; ++k) {
        if (t.dims[k] == 1) continue;
        dims[n] = t.dims[k];
        ss[n] = t.sstride[k];
        ds[n] = t.dstride[k];
        ++n;
    }
    int m = 0;
    for (int k = 0; k < n; ++k) {
        if (m > 0 && ss[m - 1] == ss[k] * dims[k] && ds[m - 1] == ds[k] * dims[k] &&
            (int64_t)dims[m - 1] * dims[k] < (1LL << 30)) {
            dims[m - 1] *= dims[k];
            ss[m - 1] = ss[k];
            ds[m - 1] = ds[k];
        } else {
            dims[m] = dims[k];
            ss[m] = ss[k];
            ds[m] = ds[k];
            ++m;
        }
    }
    if (m == 0) { m = 1; dims[0] = 1; ss[0] = 1; ds[0] = 1; }
    t.rank = m;
    for (int k = 0; k < kMaxCopyRank; ++k) {
        t.dims[k] = k < m ? dims[k] : 1;
        t.sstride[k] = k < m ? ss[k] : 0;
        t.dstride[k] = k < m ? ds[k] : 0;
    }
    // a copy whose unit-stride destination dim reads with a large source
    // stride while another dim is unit-stride in the source is transposed
    // through LDS so that both sides stay coalesced
    t.tr_in = t.tr_out = -1;
    t.lg_out = 0;
    if (t.src_buf >= 0) {
        int din = -1, dout = -1;
        for (int k = 0; k < m; ++k) {
            if (t.sstride[k] == 1) din = k;
            if (t.dstride[k] == 1) dout = k;
        }
        // tiles of 1024 elements, 16 x 64, 32 x 32 or 64 x 16 (destination-
        // contiguous x source-contiguous): the shape whose first tile leaves
        // the smallest part idle, used when that part is at most a quarter
        // (an idle part costs more than the uncoalesced reads save)
        if (din >= 0 && dout >= 0 && din != dout && t.dims[din] >= 16 && t.dims[dout] >= 16) {
            int best = -1;
            double best_used = 0.0;
            for (int lg : {5, 4, 6}) {           // 32 x 32 first: it wins ties
                const int to = 1 << lg, ti = 1024 >> lg;
                const double used = (double)std::min(to, t.dims[dout]) * std::min(ti, t.dims[din]) / 1024.0;
                if (used > best_used + 1e-12) { best = lg; best_used = used; }
            }
            if (best >= 0 && best_used >= 0.75) {
                t.tr_in = din;
                t.tr_out = dout;
                t.lg_out = best;
            }
        }
    }
}

int64_t copy_task_chunks(const CopyTask& t) {
    if (t.tr_in < 0) return (t.count + 1023) / 1024;
    const int64_t to = 1 << t.lg_out, ti = 1024 >> t.lg_out;
    int64_t n = ((t.dims[t.tr_out] + to - 1) / to) * ((t.dims[t.tr_in] + ti - 1) / ti);
    for (int k = 0; k < t.rank; ++k)
        if (k != t.tr_in && k != t.tr_out) n *= t.dims[k];
    return n;
}

CopyTask make_copy_task(int src_buf, int64_t src_off, int dst_buf, int64_t dst_off, const std::vector<int>& dims,
                        const std::vector<int64_t>& sstr, const std::vector<int64_t>& dstr, double scale) {
    CopyTask t{};
    if ((int)dims.size() > kMaxCopyRank) fail(SYMTEN_E_CAPACITY, "copy task rank exceeds 8");
    t.src_buf = src_buf;
    t.dst_buf = dst_buf;
    t.src_off = src_off;
    t.dst_off = dst_off;
    t.rank = (int)dims.size();
    int64_t c = 1;
    for (size_t k = 0; k < dims.size(); ++k) {
        t.dims[k] = dims[k];
        t.sstride[k] = src_buf >= 0 ? sstr[k] : 0;
        t.dstride[k] = dstr[k];
        c *= dims[k];
    }
    if (c >= (1LL << 31)) fail(SYMTEN_E_CAPACITY, "copy task too large");
    t.count = (int)c;
    t.scale = scale;
    simplify_task(t);
    t.nchunks = (int)copy_task_chunks(t);
    return t;
}

static std::vector<int64_t> suffix(const std::vector<int>& d, int64_t mult) {
    std::vector<int64_t> s(d.size());
    int64_t st = mult;
    for (int k = (int)d.size() - 1; k >= 0; --k) { s[k] = st; st *= d[k]; }
    return s;
}
static int64_t prod(const std::vector<int>& d) {
    int64_t p = 1;
    for (int x : d) p *= x;
    return p;
}

// -------------------------------------------------------------- planning
namespace {
struct GroupBuild {
    std::map<std::vector<int>, std::vector<int>> alpha_blocks;   // alpha -> A block ids
    std::map<std::vector<int>, std::vector<int>> beta_blocks;    // beta -> B block ids
    std::set<std::vector<int>> kapA, kapB;
};
}  // namespace

std::shared_ptr<ContractPlan> plan_contraction(const Tensor& A, const Tensor& B, int ncon, const int* legsA,
                                               const int* legsB, const int* out_perm, int prec) {
    if (A.group != B.group) fail(SYMTEN_E_SYM, "contract: operands have different symmetry groups");
    const int RA = A.rank(), RB = B.rank();
    if (ncon < 0 || ncon > RA || ncon > RB) fail(SYMTEN_E_INVAL, "contract: bad ncon");
    if (ncon > 0 && (!legsA || !legsB)) fail(SYMTEN_E_INVAL, "contract: null leg list");
    std::vector<int> conA(ncon), conB(ncon);
    std::vector<char> usedA(RA, 0), usedB(RB, 0);
    for (int i = 0; i < ncon; ++i) {
        conA[i] = legsA[i];
        conB[i] = legsB[i];
        if (conA[i] < 0 || conA[i] >= RA || conB[i] < 0 || conB[i] >= RB)
            fail(SYMTEN_E_INVAL, "contract: leg index out of range");
        if (usedA[conA[i]]++ || usedB[conB[i]]++) fail(SYMTEN_E_INVAL, "contract: leg listed twice");
        const Leg& la = A.legs[conA[i]];
        const Leg& lb = B.legs[conB[i]];
        if (la.dir != -lb.dir) fail(SYMTEN_E_LEGS, "contract: contracted legs must have opposite directions");
        if (!la.same_sectors(lb)) fail(SYMTEN_E_LEGS, "contract: contracted legs have different sectors");
    }
    Prec p;
    switch (prec) {
        case SYMTEN_PREC_F64: p = Prec::F64; break;
        case SYMTEN_PREC_F32: p = Prec::F32; break;
        case SYMTEN_PREC_BF16: p = Prec::BF16; break;
        case SYMTEN_PREC_BF16X3: p = Prec::BF16X3; break;
        case SYMTEN_PREC_BF16X6: p = Prec::BF16X6; break;
        default: fail(SYMTEN_E_INVAL, "contract: unknown precision");
    }
    if (A.dtype != B.dtype) fail(SYMTEN_E_INVAL, "contract: operands have different storage types");
    if ((p == Prec::F64) != (A.dtype == SYMTEN_F64))
        fail(SYMTEN_E_INVAL, "contract: PREC_F64 needs F64 storage, the other precisions F32 storage");

    std::vector<int> freeA, freeB;
    for (int l = 0; l < RA; ++l) if (!usedA[l]) freeA.push_back(l);
    for (int l = 0; l < RB; ++l) if (!usedB[l]) freeB.push_back(l);
    const int RO = (int)(freeA.size() + freeB.size());
    if (RO == 0) fail(SYMTEN_E_UNSUPPORTED, "contract: full contraction to a scalar");
    if (RO > SYMTEN_MAX_RANK) fail(SYMTEN_E_CAPACITY, "contract: output rank exceeds 8");
    std::vector<int> perm(RO);
    std::iota(perm.begin(), perm.end(), 0);
    if (out_perm) {
        std::vector<char> seen(RO, 0);
        for (int j = 0; j < RO; ++j) {
            perm[j] = out_perm[j];
            if (perm[j] < 0 || perm[j] >= RO || seen[perm[j]]++) fail(SYMTEN_E_INVAL, "contract: bad out_perm");
        }
    }

    if (A.group == SYMTEN_SU2) return plan_contraction_su2(A, B, conA, conB, freeA, freeB, perm, p);

    auto plan = std::make_shared<ContractPlan>();
    plan->prec = p;
    plan->panel_f64 = (p == Prec::F64);
    plan->conA = conA;
    plan->conB = conB;
    const int VW = panel_vw(p);   // 16-byte vectors in the GEMM loads

    // group blocks by the contracted charge seen from A
    const int cm = charge_mod(A.group);
    std::map<int, GroupBuild> gb;
    for (size_t i = 0; i < A.blocks.size(); ++i) {
        const Block& b = A.blocks[i];
        std::vector<int> al, ka;
        int key = 0;
        for (int l : freeA) al.push_back(b.q[l]);
        for (int l : conA) { ka.push_back(b.q[l]); key += A.legs[l].dir * b.q[l]; }
        key = cnorm(key, cm);
        GroupBuild& G = gb[key];
        G.alpha_blocks[al].push_back((int)i);
        G.kapA.insert(ka);
    }
    for (size_t i = 0; i < B.blocks.size(); ++i) {
        const Block& b = B.blocks[i];
        std::vector<int> be, ka;
        int key = 0;
        for (int l : freeB) be.push_back(b.q[l]);
        for (int l : conB) { ka.push_back(b.q[l]); key -= B.legs[l].dir * b.q[l]; }
        key = cnorm(key, cm);
        auto it = gb.find(key);
        if (it == gb.end()) continue;
        it->second.beta_blocks[be].push_back((int)i);
        it->second.kapB.insert(ka);
    }

    // output metadata
    auto out = std::make_shared<Tensor>();
    out->group = A.group;
    out->flux = cnorm(A.flux + B.flux, cm);
    out->dtype = A.dtype;
    std::vector<Leg> olegs;
    for (int l : freeA) olegs.push_back(A.legs[l]);
    for (int l : freeB) olegs.push_back(B.legs[l]);
    out->legs.resize(RO);
    for (int j = 0; j < RO; ++j) out->legs[j] = olegs[perm[j]];

    int64_t a_pos = 0, b_pos = 0, c_pos = 0;
    symten_plan_stats info{};
    auto align32 = [](int64_t x) { return (x + 31) / 32 * 32; };

    auto key_of = [](const Tensor& T, const Block& b, const std::vector<int>& legs) {
        std::vector<int> k;
        for (int l : legs) k.push_back(b.q[l]);
        return k;
    };

    for (auto& kv : gb) {
        GroupBuild& G = kv.second;
        std::vector<std::vector<int>> kap;
        for (auto& k : G.kapA) if (G.kapB.count(k)) kap.push_back(k);
        if (kap.empty()) continue;
        std::map<std::vector<int>, int> kidx;
        for (size_t i = 0; i < kap.size(); ++i) kidx[kap[i]] = (int)i;
        // kappa dims and offsets
        std::vector<int> koff(kap.size());
        std::vector<int64_t> kdim(kap.size());
        int64_t K = 0;
        for (size_t i = 0; i < kap.size(); ++i) {
            int64_t d = 1;
            for (int c = 0; c < ncon; ++c) d *= A.legs[conA[c]].dim_of(kap[i][c]);
            kdim[i] = d;
            koff[i] = (int)K;
            K += d;
        }
        // rows: alphas with at least one A block whose kappa is kept
        GroupPlan gp;
        gp.key = kv.first;
        std::vector<std::vector<int>> rows_blocks, cols_blocks;
        int64_t M = 0, N = 0;
        for (auto& ab : G.alpha_blocks) {
            std::vector<int> keep;
            for (int bi : ab.second)
                if (kidx.count(key_of(A, A.blocks[bi], conA))) keep.push_back(bi);
            if (keep.empty()) continue;
            gp.rows.push_back(ab.first);
            gp.row_off.push_back((int)M);
            int64_t d = 1;
            for (size_t c = 0; c < freeA.size(); ++c) d *= A.legs[freeA[c]].dim_of(ab.first[c]);
            M += d;
            rows_blocks.push_back(keep);
        }
        for (auto& bb : G.beta_blocks) {
            std::vector<int> keep;
            for (int bi : bb.second)
                if (kidx.count(key_of(B, B.blocks[bi], conB))) keep.push_back(bi);
            if (keep.empty()) continue;
            gp.cols.push_back(bb.first);
            gp.col_off.push_back((int)N);
            int64_t d = 1;
            for (size_t c = 0; c < freeB.size(); ++c) d *= B.legs[freeB[c]].dim_of(bb.first[c]);
            N += d;
            cols_blocks.push_back(keep);
        }
        if (M == 0 || N == 0 || K == 0) continue;
        if (M >= (1LL << 31) || N >= (1LL << 31) || K >= (1LL << 30)) fail(SYMTEN_E_CAPACITY, "contract: sector too large");
        const int64_t lda = (K + VW - 1) / VW * VW;
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
        info.max_m = std::max<int64_t>(info.max_m, M);
        info.max_n = std::max<int64_t>(info.max_n, N);
        info.max_k = std::max<int64_t>(info.max_k, K);

        // A panel tasks
        for (size_t r = 0; r < gp.rows.size(); ++r) {
            std::vector<char> present(kap.size(), 0);
            std::vector<int> adims;
            for (size_t c = 0; c < freeA.size(); ++c) adims.push_back(A.legs[freeA[c]].dim_of(gp.rows[r][c]));
            const int64_t ra = prod(adims);
            for (int bi : rows_blocks[r]) {
                const Block& b = A.blocks[bi];
                const int ki = kidx[key_of(A, b, conA)];
                present[ki] = 1;
                std::vector<int> dims, kd;
                std::vector<int64_t> ss;
                for (int l : freeA) { dims.push_back(b.shape[l]); ss.push_back(b.stride[l]); }
                for (int l : conA) { dims.push_back(b.shape[l]); ss.push_back(b.stride[l]); kd.push_back(b.shape[l]); }
                std::vector<int64_t> ds = suffix(adims, lda);
                std::vector<int64_t> dk = suffix(kd, 1);
                ds.insert(ds.end(), dk.begin(), dk.end());
                const int64_t doff = gp.a_off + gp.row_off[r] * lda + koff[ki];
                plan->copies.push_back(make_copy_task(0, b.offset, 2, doff, dims, ss, ds));
                PanelMap pm{bi, doff, std::vector<int64_t>(A.rank(), 0)};
                for (size_t c = 0; c < freeA.size(); ++c) pm.dstride[freeA[c]] = ds[c];
                for (size_t c = 0; c < conA.size(); ++c) pm.dstride[conA[c]] = ds[freeA.size() + c];
                plan->a_maps.push_back(std::move(pm));
            }
            for (size_t ki = 0; ki < kap.size(); ++ki)
                if (!present[ki])
                    plan->copies.push_back(make_copy_task(-1, 0, 2, gp.a_off + gp.row_off[r] * lda + koff[ki],
                                                     {(int)ra, (int)kdim[ki]}, {0, 0}, {lda, 1}));
        }
        if (lda > K)
            plan->copies.push_back(make_copy_task(-1, 0, 2, gp.a_off + K, {(int)M, (int)(lda - K)}, {0, 0}, {lda, 1}));
        // B panel tasks: B_g stored [N][lda] (K contiguous)
        for (size_t c = 0; c < gp.cols.size(); ++c) {
            std::vector<char> present(kap.size(), 0);
            std::vector<int> bdims;
            for (size_t x = 0; x < freeB.size(); ++x) bdims.push_back(B.legs[freeB[x]].dim_of(gp.cols[c][x]));
            const int64_t nb = prod(bdims);
            for (int bi : cols_blocks[c]) {
                const Block& b = B.blocks[bi];
                const int ki = kidx[key_of(B, b, conB)];
                present[ki] = 1;
                std::vector<int> dims, kd;
                std::vector<int64_t> ss;
                for (int l : freeB) { dims.push_back(b.shape[l]); ss.push_back(b.stride[l]); }
                for (int l : conB) { dims.push_back(b.shape[l]); ss.push_back(b.stride[l]); kd.push_back(b.shape[l]); }
                std::vector<int64_t> ds = suffix(bdims, lda);
                std::vector<int64_t> dk = suffix(kd, 1);
                ds.insert(ds.end(), dk.begin(), dk.end());
                plan->copies.push_back(make_copy_task(1, b.offset, 3, gp.b_off + gp.col_off[c] * lda + koff[ki], dims, ss, ds));
            }
            for (size_t ki = 0; ki < kap.size(); ++ki)
                if (!present[ki])
                    plan->copies.push_back(make_copy_task(-1, 0, 3, gp.b_off + gp.col_off[c] * lda + koff[ki],
                                                     {(int)nb, (int)kdim[ki]}, {0, 0}, {lda, 1}));
        }
        if (lda > K)
            plan->copies.push_back(make_copy_task(-1, 0, 3, gp.b_off + K, {(int)N, (int)(lda - K)}, {0, 0}, {lda, 1}));

        // output blocks reached by at least one pair; pair statistics
        std::vector<std::vector<char>> arow(gp.rows.size(), std::vector<char>(kap.size(), 0));
        std::vector<std::vector<char>> bcol(gp.cols.size(), std::vector<char>(kap.size(), 0));
        for (size_t r = 0; r < gp.rows.size(); ++r)
            for (int bi : rows_blocks[r]) arow[r][kidx[key_of(A, A.blocks[bi], conA)]] = 1;
        for (size_t c = 0; c < gp.cols.size(); ++c)
            for (int bi : cols_blocks[c]) bcol[c][kidx[key_of(B, B.blocks[bi], conB)]] = 1;
        for (size_t r = 0; r < gp.rows.size(); ++r) {
            std::vector<int> adims;
            for (size_t c = 0; c < freeA.size(); ++c) adims.push_back(A.legs[freeA[c]].dim_of(gp.rows[r][c]));
            const int64_t ma = prod(adims);
            for (size_t c = 0; c < gp.cols.size(); ++c) {
                int64_t npairs = 0, fl = 0;
                std::vector<int> bdims;
                for (size_t x = 0; x < freeB.size(); ++x) bdims.push_back(B.legs[freeB[x]].dim_of(gp.cols[c][x]));
                const int64_t nbd = prod(bdims);
                for (size_t ki = 0; ki < kap.size(); ++ki)
                    if (arow[r][ki] && bcol[c][ki]) { ++npairs; fl += 2 * ma * nbd * kdim[ki]; }
                if (!npairs) continue;
                info.pairs += npairs;
                info.useful_flops += fl;
                info.out_blocks += 1;
                Block ob;
                std::vector<int> q = gp.rows[r];
                q.insert(q.end(), gp.cols[c].begin(), gp.cols[c].end());
                std::vector<int> shp = adims;
                shp.insert(shp.end(), bdims.begin(), bdims.end());
                std::vector<int64_t> st = suffix(adims, N);
                std::vector<int64_t> sb = suffix(bdims, 1);
                st.insert(st.end(), sb.begin(), sb.end());
                ob.q.resize(RO);
                ob.shape.resize(RO);
                ob.stride.resize(RO);
                for (int j = 0; j < RO; ++j) {
                    ob.q[j] = q[perm[j]];
                    ob.shape[j] = shp[perm[j]];
                    ob.stride[j] = st[perm[j]];
                }
                ob.offset = gp.c_off + gp.row_off[r] * N + gp.col_off[c];
                ob.size = ma * nbd;
                out->blocks.push_back(std::move(ob));
            }
        }
        plan->groups.push_back(std::move(gp));
    }
    std::sort(out->blocks.begin(), out->blocks.end(), [](const Block& x, const Block& y) { return x.q < y.q; });
    out->rebuild_index();
    out->elems = c_pos;
    out->meta_only = true;
    plan->out_meta = out;
    plan->a_panel_elems = a_pos;
    plan->b_panel_elems = b_pos;
    plan->out_elems = c_pos;
    plan->info = info;
    if (panel_planes(p) > 1)   // each lower plane follows the whole plane above it
        for (auto& t : plan->copies) t.lo_off = t.dst_buf == 2 ? a_pos : b_pos;
    return plan;
}

// -------------------------------------------------------------- execution
// -------------------------------------------------------------- profiling
namespace {
struct ProfRec {
    std::string name;
    int64_t uf, gf, bytes;
    hipEvent_t a, b;
};
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<ProfRec> recs;
};
}  // namespace
Profiler& profiler() {
    static Profiler* p = new Profiler();
    return *p;
}
bool profiling() { return profiler().on; }

void profile_launch(const std::string& name, int64_t uf, int64_t gf, int64_t bytes, hipStream_t s,
                    const std::function<void()>& launch) {
    Profiler& P = profiler();
    if (!P.on) { launch(); return; }
    ProfRec r{name, uf, gf, bytes, nullptr, nullptr};
    HIPCHK(hipEventCreate(&r.a));
    HIPCHK(hipEventCreate(&r.b));
    HIPCHK(hipEventRecord(r.a, s));
    launch();
    HIPCHK(hipEventRecord(r.b, s));
    std::lock_guard<std::mutex> lk(P.mu);
    P.recs.push_back(r);
}

void profile_begin() {
    Profiler& P = profiler();
    std::lock_guard<std::mutex> lk(P.mu);
    for (auto& r : P.recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    P.recs.clear();
    P.on = true;
}

std::vector<symten_kernel_stat> profile_end() {
    Profiler& P = profiler();
    std::lock_guard<std::mutex> lk(P.mu);
    P.on = false;
    std::map<std::string, symten_kernel_stat> agg;
    for (auto& r : P.recs) {
        HIPCHK(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        symten_kernel_stat& k = agg[r.name];
        std::snprintf(k.name, sizeof(k.name), "%s", r.name.c_str());
        k.launches += 1;
        k.ms += ms;
        k.useful_flops += r.uf;
        k.gemm_flops += r.gf;
        k.bytes += r.bytes;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    P.recs.clear();
    std::vector<symten_kernel_stat> out;
    for (auto& kv : agg) out.push_back(kv.second);
    return out;
}

std::string gemm_kernel_name(Prec p, int cfg, bool scatter) {
    const std::string t = std::to_string(gemm_tile_bm(p, cfg)) + "x" + std::to_string(gemm_tile_bn(p, cfg)) + "x" +
                          std::to_string(gemm_tile_bk(p, cfg));
    const std::string sc = scatter ? ",scatter" : "";
    switch (p) {
        case Prec::F64: return "gemm_f64_kernel<" + t + ">";
        case Prec::F32: return "gemm_f32_kernel<" + t + ",f32>";
        case Prec::BF16: return "gemm_bf16_kernel<" + t + ",bf16" + sc + ">";
        case Prec::BF16X3: return "gemm_bf16_kernel<" + t + ",bf16x3" + sc + ">";
        default: return "gemm_bf16_kernel<" + t + ",bf16x6" + sc + ">";
    }
}

int64_t copy_bytes(const std::vector<CopyTask>& tasks, size_t se, size_t de) {
    int64_t b = 0;
    for (auto& t : tasks) b += (int64_t)t.count * ((t.src_buf >= 0 ? se : 0) + de);
    return b;
}

int64_t gemm_bytes(const std::vector<GemmGroup>& gs, size_t pe, size_t oe) {
    int64_t b = 0;
    for (auto& g : gs) b += (int64_t)pe * ((int64_t)g.M * g.K + (int64_t)g.N * g.K) + (int64_t)oe * g.M * g.N;
    return b;
}

namespace {
// Device copies of a plan's descriptors, uploaded once per plan.
struct DevPlan {
    BufferPtr tasks, prefix, groups;
    int ntasks = 0;
    int64_t npieces = 0;
    TileChoice tc;
    std::vector<GemmGroup> host_groups;
    int64_t checked_a = -1, checked_b = -1;   // input sizes already validated
};
std::mutex g_devplan_mu;
}  // namespace

void upload_sync(BufferPtr& buf, const void* host, size_t bytes) {
    buf = device_alloc(bytes);
    if (bytes) HIPCHK(hipMemcpy(buf->ptr, host, bytes, hipMemcpyHostToDevice));
}

// ---------------------------------------------------------------- autotuner
namespace {
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;   // shape signature -> tile configuration
bool g_tune_loaded = false;

std::string shape_key(const std::vector<GemmGroup>& groups, Prec prec) {
    // the epilogue kind is part of the shape: a scatter epilogue is another kernel
    std::string k = "p" + std::to_string((int)prec) + ":";
    for (auto& g : groups)
        k += std::to_string(g.M) + "x" + std::to_string(g.N) + "x" + std::to_string(g.K) + (g.scatter ? "s," : ",");
    char h[32];
    std::snprintf(h, sizeof(h), "%016zx", std::hash<std::string>{}(k));
    return std::string(h) + "/" + std::to_string(groups.size());
}

// Decisions persist across processes when SYMTEN_TUNE_CACHE names a file.
void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("SYMTEN_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[128];
    int cfg;
    while (std::fscanf(f, "%127s %d", key, &cfg) == 2) g_tune[key] = cfg;
    std::fclose(f);
}
void tune_store_locked(const std::string& key, int cfg) {
    g_tune[key] = cfg;
    const char* path = std::getenv("SYMTEN_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d\n", key.c_str(), cfg);
    std::fclose(f);
}
}  // namespace

void ensure_tiles(TileChoice& tc, const std::vector<GemmGroup>& groups, Prec prec, int cfg) {
    if (tc.tiles[cfg]) return;
    TilePlan tp;
    build_tiles(groups, prec, cfg, tp, true);
    tc.ntiles[cfg] = (int)tp.tiles.size();
    upload_sync(tc.tiles[cfg], tp.tiles.data(), tp.tiles.size() * sizeof(TileWork));
    tc.nsplits[cfg] = (int)tp.splits.size();
    if (!tp.splits.empty()) upload_sync(tc.splits[cfg], tp.splits.data(), tp.splits.size() * sizeof(SplitOut));
    const bool persistent = gemm_persistent(tc.ntiles[cfg], gemm_capacity(prec, cfg));
    tc.ws_bytes[cfg] = tp.partial_tiles * gemm_tile_bm(prec, cfg) * gemm_tile_bn(prec, cfg) *
                           (prec == Prec::F64 ? 8 : 4) +
                       (persistent || tp.partial_tiles ? kSplitQueueBytes : 0);
}

void autotune_gemm(TileChoice& tc, const std::vector<GemmGroup>& groups, Prec prec,
                   const std::function<void(int)>& launch, hipStream_t s) {
    if (tc.cfg >= 0) return;
    int maxm = 0, maxn = 0;
    for (auto& g : groups) { maxm = std::max(maxm, g.M); maxn = std::max(maxn, g.N); }
    const int heuristic = (maxm >= 128 && maxn >= 128) ? 1 : 0;
    const char* forced = std::getenv("SYMTEN_TILE_CFG");
    if (forced && *forced) {
        const int c = std::atoi(forced);
        tc.cfg = gemm_tile_ok(prec, c) ? c : heuristic;
        ensure_tiles(tc, groups, prec, tc.cfg);
        return;
    }
    const std::string key = shape_key(groups, prec);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end() && gemm_tile_ok(prec, it->second)) {
            tc.cfg = it->second;
            ensure_tiles(tc, groups, prec, tc.cfg);
            return;
        }
    }
    const char* off = std::getenv("SYMTEN_AUTOTUNE");
    if (off && std::string(off) == "0") {
        tc.cfg = heuristic;
        ensure_tiles(tc, groups, prec, tc.cfg);
        return;
    }
    hipEvent_t e[3];
    for (auto& x : e) HIPCHK(hipEventCreate(&x));
    int best = -1;
    float best_ms = 0.f;
    for (int c = 0; c < kNumTileCfg; ++c) {
        if (!gemm_tile_ok(prec, c)) continue;
        ensure_tiles(tc, groups, prec, c);
        HIPCHK(hipEventRecord(e[0], s));
        launch(c);   // first run: code-object load, caches
        HIPCHK(hipEventRecord(e[1], s));
        launch(c);
        HIPCHK(hipEventRecord(e[2], s));
        HIPCHK(hipEventSynchronize(e[2]));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e[1], e[2]));
        tc.ms[c] = ms;
        if (best < 0 || ms < best_ms) { best = c; best_ms = ms; }
    }
    for (auto& x : e) (void)hipEventDestroy(x);
    tc.cfg = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_store_locked(key, best);
}

int choose_tile_cfg(const ContractPlan& p) {
    // large tiles once the biggest sector fills them
    return (p.info.max_m >= 128 && p.info.max_n >= 128) ? 1 : 0;
}

// Work list of one grouped-GEMM launch, laid out for the 8 XCDs of the chip.
// Workgroups are dispatched to the XCDs round robin (workgroup p runs on XCD
// p mod 8; the persistent grid is a multiple of 8, so the workgroup that
// walks entries p, p + G, ... stays on one XCD), and each XCD has its own
// L2, so the tiles that share operand panels are kept on one XCD: every
// group (or, for a group heavier than an eighth of the launch, a contiguous
// range of its tile rows) goes to one XCD, the XCDs are balanced by greedy
// longest-first assignment of the work (tiles x K), each XCD's list runs
// longest K first, and the lists are interleaved with no-op entries (group
// -1) padding the shorter ones.
//
// Split K: when the launch has fewer output tiles than the chip holds
// workgroups at once, the tiles of groups with a long K are cut into parts
// of at least four K stages (s parts, s <= 8, about enough to fill the chip),
// each part writing a partial tile to its own workspace slot; a second
// kernel adds the parts of every tile in part order (deterministic).
void build_tiles(const std::vector<GemmGroup>& groups, Prec prec, int cfg, TilePlan& tp, bool allow_split) {
    constexpr int kXcd = 8;
    const int BM = gemm_tile_bm(prec, cfg), BN = gemm_tile_bn(prec, cfg), BK = gemm_tile_bk(prec, cfg);
    struct Item { int group, r0, r1; double work; };
    double total = 0.0;
    int64_t ntile = 0;
    for (auto& g : groups) {
        const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
        total += (double)tm * tn * g.K;
        ntile += (int64_t)tm * tn;
    }
    // parts per tile of each group (1: no split)
    std::vector<int> parts_of(groups.size(), 1);
    if (allow_split && ntile > 0) {
        const int64_t cap = gemm_capacity(prec, cfg);
        const int want = (int)std::min<int64_t>(8, cap / ntile);
        if (want >= 2)
            for (size_t gi = 0; gi < groups.size(); ++gi)
                parts_of[gi] = groups[gi].scatter ? 1 : std::max(1, std::min(want, groups[gi].K / (4 * BK)));
    }
    const double target = total / kXcd;
    std::vector<Item> items;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const GemmGroup& g = groups[gi];
        const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
        const double row_work = (double)tn * g.K;
        const double w = row_work * tm;
        const int parts = target > 0 ? std::max(1, std::min(tm, (int)std::ceil(w / target))) : 1;
        for (int p = 0; p < parts; ++p) {
            const int r0 = (int)((int64_t)tm * p / parts), r1 = (int)((int64_t)tm * (p + 1) / parts);
            if (r1 > r0) items.push_back({(int)gi, r0, r1, row_work * (r1 - r0)});
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.work > b.work; });
    std::vector<std::vector<Item>> bin(kXcd);
    std::vector<double> load(kXcd, 0.0);
    for (auto& it : items) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        bin[x].push_back(it);
        load[x] += it.work;
    }
    std::vector<std::vector<TileWork>> lists(kXcd);
    size_t longest = 0;
    int slot = 0;
    for (int x = 0; x < kXcd; ++x) {
        // longest K first inside the XCD so that the heaviest tiles start early
        std::stable_sort(bin[x].begin(), bin[x].end(),
                         [&](const Item& a, const Item& b) { return groups[a.group].K > groups[b.group].K; });
        for (auto& it : bin[x]) {
            const GemmGroup& g = groups[it.group];
            const int tn = (g.N + BN - 1) / BN;
            const int s = parts_of[it.group];
            // K parts of equal whole stages; the last one ends at K
            const int stages = (g.K + BK - 1) / BK;
            for (int i = it.r0; i < it.r1; ++i)
                for (int j = 0; j < tn; ++j) {
                    if (s == 1) {
                        lists[x].push_back(TileWork{it.group, i, j, 0, g.K, -1, 0, 0});
                        continue;
                    }
                    tp.splits.push_back(SplitOut{it.group, i, j, slot, s, 0});
                    for (int p = 0; p < s; ++p) {
                        const int k0 = (int)((int64_t)stages * p / s) * BK;
                        const int k1 = p + 1 == s ? g.K : (int)((int64_t)stages * (p + 1) / s) * BK;
                        lists[x].push_back(TileWork{it.group, i, j, k0, k1, slot + p, 0, 0});
                    }
                    slot += s;
                }
        }
        longest = std::max(longest, lists[x].size());
    }
    tp.partial_tiles = slot;
    tp.tiles.reserve(tp.tiles.size() + longest * kXcd);
    for (size_t i = 0; i < longest; ++i)
        for (int x = 0; x < kXcd; ++x)
            tp.tiles.push_back(i < lists[x].size() ? lists[x][i] : TileWork{-1, 0, 0, 0, 0, -1, 0, 0});
}

void copy_prefix(const std::vector<CopyTask>& tasks, std::vector<int64_t>& prefix) {
    prefix.resize(tasks.size() + 1);
    prefix[0] = 0;
    for (size_t i = 0; i < tasks.size(); ++i)
        prefix[i + 1] = prefix[i] + (copy_task_chunks(tasks[i]) + kCopyGroup - 1) / kCopyGroup;
}

// Every element a task or a GEMM group touches must lie inside its buffer;
// checked on the host before any descriptor reaches the device.
void validate_tasks(const std::vector<CopyTask>& tasks, const std::vector<int64_t>& buf_elems, int planes) {
    for (const CopyTask& t : tasks) {
        int64_t smax = t.src_off, dmax = t.dst_off, smin = t.src_off, dmin = t.dst_off;
        for (int k = 0; k < t.rank; ++k) {
            if (t.dims[k] < 1) fail(SYMTEN_E_INVAL, "internal: copy task with empty dim");
            const int64_t ds = (int64_t)(t.dims[k] - 1) * t.dstride[k];
            const int64_t ss = (int64_t)(t.dims[k] - 1) * t.sstride[k];
            (ds >= 0 ? dmax : dmin) += ds;
            (ss >= 0 ? smax : smin) += ss;
        }
        // split panels also write (planes - 1) * lo_off elements further (the lower planes)
        if (t.dst_buf < 0 || t.dst_buf >= (int)buf_elems.size() || dmin < 0 || t.lo_off < 0 || planes < 1 ||
            dmax + (planes - 1) * t.lo_off >= buf_elems[t.dst_buf])
            fail(SYMTEN_E_INVAL, "internal: copy destination out of bounds");
        if (t.src_buf >= 0 && (t.src_buf >= (int)buf_elems.size() || smin < 0 || smax >= buf_elems[t.src_buf]))
            fail(SYMTEN_E_INVAL, "internal: copy source out of bounds");
        if (t.nextra < 0 || t.nextra > kMaxExtraSrc || (t.nextra > 0 && t.src_buf < 0))
            fail(SYMTEN_E_INVAL, "internal: bad extra source count");
        if (t.nchunks != copy_task_chunks(t)) fail(SYMTEN_E_INVAL, "internal: copy task chunk count");
        if (t.tr_in >= 0 && (t.src_buf < 0 || t.tr_in >= t.rank || t.tr_out < 0 || t.tr_out >= t.rank ||
                             t.tr_in == t.tr_out || t.lg_out < 4 || t.lg_out > 6))
            fail(SYMTEN_E_INVAL, "internal: bad transposing copy tile");
        for (int x = 0; x < t.nextra; ++x) {
            const int64_t lo = smin - t.src_off + t.xsrc_off[x], hi = smax - t.src_off + t.xsrc_off[x];
            if (lo < 0 || hi >= buf_elems[t.src_buf]) fail(SYMTEN_E_INVAL, "internal: extra copy source out of bounds");
        }
    }
}

void validate_groups(const std::vector<GemmGroup>& groups, const std::vector<int64_t>& buf_elems, int vw,
                     int planes) {
    for (const GemmGroup& g : groups) {
        auto in = [&](int b, int64_t off, int64_t n) {
            return b >= 0 && b < (int)buf_elems.size() && off >= 0 && off + n <= buf_elems[b];
        };
        if (g.M < 1 || g.N < 1 || g.K < 1 || g.lda < g.K || g.ldb < g.K || g.ldc < g.N || g.lda % vw ||
            g.ldb % vw || g.a_off % vw || g.b_off % vw)
            fail(SYMTEN_E_INVAL, "internal: GEMM group shape or alignment");
        // a scatter group's destinations are checked with its tables (validate_scatter)
        const bool c_ok = g.scatter ? (g.scatter == 1 && g.c_buf >= 0 && g.c_buf < (int)buf_elems.size() &&
                                       g.s_buf >= 0 && g.s_buf < (int)buf_elems.size())
                                    : in(g.c_buf, g.c_off, (int64_t)(g.M - 1) * g.ldc + g.N);
        if (!in(g.a_buf, g.a_off, (int64_t)g.M * g.lda) || !in(g.b_buf, g.b_off, (int64_t)g.N * g.ldb) || !c_ok)
            fail(SYMTEN_E_INVAL, "internal: GEMM operand out of bounds");
        for (int p = 1; p < planes; ++p)
            if (g.a_lo % vw || g.b_lo % vw || g.a_lo < 0 || g.b_lo < 0 ||
                !in(g.a_buf, g.a_off + p * g.a_lo, (int64_t)g.M * g.lda) ||
                !in(g.b_buf, g.b_off + p * g.b_lo, (int64_t)g.N * g.ldb))
                fail(SYMTEN_E_INVAL, "internal: GEMM lower plane out of bounds");
    }
}

int64_t append_scatter_tables(const ContractPlan& p, const Tensor& A, const Tensor& B, const ContractPlan& q,
                              int64_t a_base, GemmGroup* groups, std::vector<int>& tab) {
    const Tensor& out = *p.out_meta;
    std::vector<int> map_of(out.blocks.size(), -1);
    for (size_t m = 0; m < q.a_maps.size(); ++m) {
        const int b = q.a_maps[m].block;
        if (b < 0 || b >= (int)out.blocks.size() || map_of[b] >= 0 ||
            (int)q.a_maps[m].dstride.size() != out.rank())
            fail(SYMTEN_E_INVAL, "internal: scatter tables: bad block map");
        map_of[b] = (int)m;
    }
    std::vector<int> freeA, freeB;
    for (int l = 0; l < A.rank(); ++l)
        if (std::find(p.conA.begin(), p.conA.end(), l) == p.conA.end()) freeA.push_back(l);
    for (int l = 0; l < B.rank(); ++l)
        if (std::find(p.conB.begin(), p.conB.end(), l) == p.conB.end()) freeB.push_back(l);
    const int nr = (int)freeA.size(), nc = (int)freeB.size();
    if (nr > kScatterLegs || nc > kScatterLegs || nr + nc != out.rank())
        fail(SYMTEN_E_INVAL, "internal: scatter tables: more free legs than the epilogue decodes");
    auto dims_of = [](const Tensor& T, const std::vector<int>& legs, const std::vector<int>& key) {
        std::vector<int> d;
        for (size_t c = 0; c < legs.size(); ++c) d.push_back(T.legs[legs[c]].dim_of(key[c]));
        return d;
    };
    // one entry per row (column): its block and its multi-index, row-major
    // over the block's free legs
    auto entries = [&](const std::vector<int>& d, int blk, int nlegs) {
        int64_t cnt = 1;
        for (int x : d) cnt *= x;
        for (int64_t e = 0; e < cnt; ++e) {
            int idx[kScatterLegs] = {0, 0, 0};
            int64_t rest = e;
            for (int l = nlegs - 1; l >= 0; --l) {
                idx[l] = (int)(rest % d[l]);
                rest /= d[l];
            }
            tab.insert(tab.end(), {blk, idx[0], idx[1], idx[2]});
        }
    };
    int64_t written = 0;
    for (size_t gi = 0; gi < p.groups.size(); ++gi) {
        const GroupPlan& gp = p.groups[gi];
        GemmGroup& G = groups[gi];
        if (G.M != gp.M || G.N != gp.N) fail(SYMTEN_E_INVAL, "internal: scatter tables: group mismatch");
        G.s_rows = (int64_t)tab.size();
        for (size_t r = 0; r < gp.rows.size(); ++r) entries(dims_of(A, freeA, gp.rows[r]), (int)r, nr);
        G.s_cols = (int64_t)tab.size();
        for (size_t c = 0; c < gp.cols.size(); ++c) entries(dims_of(B, freeB, gp.cols[c]), (int)c, nc);
        if ((int64_t)tab.size() - G.s_rows != 4 * ((int64_t)G.M + G.N))
            fail(SYMTEN_E_INVAL, "internal: scatter tables: row or column count");
        G.s_blocks = (int64_t)tab.size();
        for (size_t r = 0; r < gp.rows.size(); ++r)
            for (size_t c = 0; c < gp.cols.size(); ++c) {
                std::vector<int> key = gp.rows[r];
                key.insert(key.end(), gp.cols[c].begin(), gp.cols[c].end());
                auto it = out.index.find(key);
                const int m = it == out.index.end() ? -1 : map_of[it->second];
                if (m < 0) {   // a block the next contraction does not read
                    tab.insert(tab.end(), {-1, 0, 0, 0, 0, 0, 0, 0});
                    continue;
                }
                const PanelMap& pm = q.a_maps[m];
                const int64_t d0 = a_base + pm.dst_off;
                if (d0 >= (1LL << 31)) fail(SYMTEN_E_CAPACITY, "scatter epilogue: A panels beyond 2^31 elements");
                int sr[kScatterLegs] = {0, 0, 0}, sc[kScatterLegs] = {0, 0, 0};
                for (int l = 0; l < nr; ++l) sr[l] = (int)pm.dstride[l];
                for (int l = 0; l < nc; ++l) sc[l] = (int)pm.dstride[nr + l];
                tab.insert(tab.end(), {(int)d0, sr[0], sr[1], sr[2], sc[0], sc[1], sc[2], 0});
                written += out.blocks[it->second].size;
            }
        G.scatter = 1;
        G.s_ncb = (int)gp.cols.size();
        G.c_off = 0;
    }
    return written;
}

void validate_scatter(const std::vector<GemmGroup>& groups, const std::vector<int>& tab, int64_t dst_elems,
                      int planes) {
    const int64_t nt = (int64_t)tab.size();
    for (const GemmGroup& g : groups) {
        if (!g.scatter) continue;
        if (g.s_ncb < 1 || g.s_rows < 0 || g.s_cols < 0 || g.s_blocks < 0 || g.s_rows % 4 || g.s_cols % 4 ||
            g.s_blocks % 4 || g.s_rows + 4 * (int64_t)g.M > nt || g.s_cols + 4 * (int64_t)g.N > nt || g.c_lo < 0)
            fail(SYMTEN_E_INVAL, "internal: scatter tables out of bounds");
        int nrb = 0;   // row blocks
        for (int i = 0; i < g.M; ++i) {
            const int* r = &tab[g.s_rows + 4 * i];
            if (r[0] < 0 || r[1] < 0 || r[2] < 0 || r[3] < 0) fail(SYMTEN_E_INVAL, "internal: scatter row entry");
            nrb = std::max(nrb, r[0] + 1);
        }
        for (int j = 0; j < g.N; ++j) {
            const int* c = &tab[g.s_cols + 4 * j];
            if (c[0] < 0 || c[0] >= g.s_ncb || c[1] < 0 || c[2] < 0 || c[3] < 0)
                fail(SYMTEN_E_INVAL, "internal: scatter column entry");
        }
        if (g.s_blocks + 8 * (int64_t)nrb * g.s_ncb > nt) fail(SYMTEN_E_INVAL, "internal: scatter block table out of bounds");
        auto entry = [&](int rb, int cb) { return &tab[g.s_blocks + 8 * ((int64_t)rb * g.s_ncb + cb)]; };
        // the largest row term and column term each block entry meets
        const size_t nb = (size_t)nrb * g.s_ncb;
        std::vector<int64_t> rmax(nb, 0), cmax(nb, 0);
        for (int i = 0; i < g.M; ++i) {
            const int* r = &tab[g.s_rows + 4 * i];
            for (int cb = 0; cb < g.s_ncb; ++cb) {
                const int* b = entry(r[0], cb);
                const size_t e = (size_t)r[0] * g.s_ncb + cb;
                rmax[e] = std::max(rmax[e], (int64_t)r[1] * b[1] + (int64_t)r[2] * b[2] + (int64_t)r[3] * b[3]);
            }
        }
        for (int j = 0; j < g.N; ++j) {
            const int* c = &tab[g.s_cols + 4 * j];
            for (int rb = 0; rb < nrb; ++rb) {
                const int* b = entry(rb, c[0]);
                const size_t e = (size_t)rb * g.s_ncb + c[0];
                cmax[e] = std::max(cmax[e], (int64_t)c[1] * b[4] + (int64_t)c[2] * b[5] + (int64_t)c[3] * b[6]);
            }
        }
        for (int rb = 0; rb < nrb; ++rb)
            for (int cb = 0; cb < g.s_ncb; ++cb) {
                const int* b = entry(rb, cb);
                if (b[0] < 0) continue;
                for (int k = 1; k < 7; ++k)
                    if (b[k] < 0) fail(SYMTEN_E_INVAL, "internal: negative scatter stride");
                const size_t e = (size_t)rb * g.s_ncb + cb;
                const int64_t top = b[0] + rmax[e] + cmax[e];
                if (top >= (1LL << 31) || top + (planes - 1) * g.c_lo >= dst_elems)
                    fail(SYMTEN_E_INVAL, "internal: scatter destination out of bounds");
            }
    }
}

static std::shared_ptr<DevPlan> dev_plan(const ContractPlan& p) {
    std::lock_guard<std::mutex> lk(g_devplan_mu);
    if (p.dev) return std::static_pointer_cast<DevPlan>(p.dev);
    auto d = std::make_shared<DevPlan>();
    std::vector<int64_t> prefix;
    copy_prefix(p.copies, prefix);
    d->ntasks = (int)p.copies.size();
    d->npieces = prefix.back();
    upload_sync(d->tasks, p.copies.data(), p.copies.size() * sizeof(CopyTask));
    upload_sync(d->prefix, prefix.data(), prefix.size() * sizeof(int64_t));
    std::vector<GemmGroup> gg;
    for (auto& g : p.groups) {
        GemmGroup x{};
        x.a_off = g.a_off;
        x.b_off = g.b_off;
        x.c_off = g.c_off;
        x.M = g.M;
        x.N = g.N;
        x.K = g.K;
        x.lda = g.lda;
        x.ldb = g.lda;
        x.ldc = g.N;
        x.a_buf = 0;
        x.b_buf = 1;
        x.c_buf = 2;
        if (panel_planes(p.prec) > 1) {
            x.a_lo = p.a_panel_elems;
            x.b_lo = p.b_panel_elems;
        }
        gg.push_back(x);
    }
    const int pl = panel_planes(p.prec);
    validate_groups(gg, {pl * p.a_panel_elems, pl * p.b_panel_elems, p.out_elems}, panel_vw(p.prec), pl);
    d->host_groups = gg;
    upload_sync(d->groups, gg.data(), gg.size() * sizeof(GemmGroup));
    p.dev = d;
    return d;
}

TensorPtr run_contraction(const ContractPlan& p, const Tensor& A, const Tensor& B, hipStream_t stream) {
    check_device_tensor(A, "contract(A)");
    check_device_tensor(B, "contract(B)");
    auto out = std::make_shared<Tensor>(*p.out_meta);
    out->meta_only = false;
    out->buf = device_alloc(std::max<int64_t>(p.out_elems, 1) * out->esize());
    if (p.groups.empty()) return out;
    auto d = dev_plan(p);
    const int pl = panel_planes(p.prec);
    if (d->checked_a != A.elems || d->checked_b != B.elems) {
        validate_tasks(p.copies, {A.elems, B.elems, pl * p.a_panel_elems, pl * p.b_panel_elems}, pl);
        d->checked_a = A.elems;
        d->checked_b = B.elems;
    }
    const size_t pe = panel_esize(p.prec) * pl;   // bytes per panel element, all planes
    BufferPtr pa = device_alloc(std::max<int64_t>(p.a_panel_elems, 1) * pe);
    BufferPtr pb = device_alloc(std::max<int64_t>(p.b_panel_elems, 1) * pe);
    const bool src64 = A.dtype == SYMTEN_F64;
    const size_t se = src64 ? 8 : 4;
    const bool prof = profiling();
    profile_launch(copy_kernel_name(src64, p.prec), 0, 0, prof ? copy_bytes(p.copies, se, pe) : 0, stream, [&] {
        copy_launch_arg((const CopyTask*)d->tasks->ptr, (const int64_t*)d->prefix->ptr, d->ntasks, d->npieces,
                        {A.data(), B.data(), pa->ptr, pb->ptr}, src64, panel_dst_kind(p.prec), stream);
    });
    auto launch = [&](int cfg) {
        const TileChoice& tc = d->tc;
        BufferPtr ws = tc.ws_bytes[cfg] ? device_alloc(tc.ws_bytes[cfg]) : nullptr;   // split-K partials
        gemm_launch_arg((const TileWork*)tc.tiles[cfg]->ptr, tc.ntiles[cfg], (const GemmGroup*)d->groups->ptr,
                        {pa->ptr, pb->ptr, out->data()}, p.prec, cfg, stream, tc.split(cfg, ws ? ws->ptr : nullptr));
    };
    autotune_gemm(d->tc, d->host_groups, p.prec, launch, stream);
    const int cfg = d->tc.cfg;
    profile_launch(gemm_kernel_name(p.prec, cfg), p.info.useful_flops, p.info.gemm_flops,
                   prof ? gemm_bytes(d->host_groups, pe, out->esize()) : 0, stream, [&] { launch(cfg); });
    // pa/pb return to the pool here; later users are ordered on the same stream
    return out;
}

// ---------------------------------------------- several contractions at once
// Independent contractions share one gather launch and one grouped-GEMM
// launch: their copy tasks and GEMM groups are concatenated once per plan
// combination, with buffer indices [A_0..A_n-1, B_0..B_n-1, A panels,
// B panels, C_0..C_n-1] passed by value to the kernels.
namespace {
struct MultiDesc {
    std::vector<std::shared_ptr<ContractPlan>> plans;   // keeps the plans alive
    BufferPtr tasks, prefix, groups;
    int ntasks = 0;
    int64_t npieces = 0, ap = 0, bp = 0;
    TileChoice tc;
    std::vector<CopyTask> host_tasks;
    std::vector<GemmGroup> host_groups;
    symten_plan_stats info{};
    std::vector<int64_t> checked;   // buffer sizes already validated
};
std::mutex g_multi_mu;
std::map<std::vector<const ContractPlan*>, std::shared_ptr<MultiDesc>> g_multi;

std::shared_ptr<MultiDesc> multi_desc(const std::vector<std::shared_ptr<ContractPlan>>& plans) {
    std::vector<const ContractPlan*> key;
    for (auto& p : plans) key.push_back(p.get());
    std::lock_guard<std::mutex> lk(g_multi_mu);
    auto it = g_multi.find(key);
    if (it != g_multi.end()) return it->second;
    const int n = (int)plans.size();
    auto d = std::make_shared<MultiDesc>();
    d->plans = plans;
    for (int i = 0; i < n; ++i) {
        const ContractPlan& p = *plans[i];
        const int64_t a0 = d->ap, b0 = d->bp;
        d->ap += (p.a_panel_elems + 31) / 32 * 32;
        d->bp += (p.b_panel_elems + 31) / 32 * 32;
        for (CopyTask t : p.copies) {
            if (t.src_buf == 0) t.src_buf = i;
            else if (t.src_buf == 1) t.src_buf = n + i;
            if (t.dst_buf == 2) { t.dst_buf = 2 * n; t.dst_off += a0; }
            else { t.dst_buf = 2 * n + 1; t.dst_off += b0; }
            d->host_tasks.push_back(t);
        }
        for (auto& g : p.groups) {
            GemmGroup x{};
            x.a_off = g.a_off + a0;
            x.b_off = g.b_off + b0;
            x.c_off = g.c_off;
            x.M = g.M;
            x.N = g.N;
            x.K = g.K;
            x.lda = x.ldb = g.lda;
            x.ldc = g.N;
            x.a_buf = 2 * n;
            x.b_buf = 2 * n + 1;
            x.c_buf = 2 * n + 2 + i;
            d->host_groups.push_back(x);
        }
        d->info.pairs += p.info.pairs;
        d->info.useful_flops += p.info.useful_flops;
        d->info.gemm_flops += p.info.gemm_flops;
        d->info.max_m = std::max(d->info.max_m, p.info.max_m);
        d->info.max_n = std::max(d->info.max_n, p.info.max_n);
    }
    if (panel_planes(plans[0]->prec) > 1) {   // the lower planes follow the concatenated hi planes
        for (auto& t : d->host_tasks) t.lo_off = t.dst_buf == 2 * n ? d->ap : d->bp;
        for (auto& g : d->host_groups) {
            g.a_lo = d->ap;
            g.b_lo = d->bp;
        }
    }
    std::vector<int64_t> prefix;
    copy_prefix(d->host_tasks, prefix);
    d->ntasks = (int)d->host_tasks.size();
    d->npieces = prefix.back();
    upload_sync(d->tasks, d->host_tasks.data(), d->host_tasks.size() * sizeof(CopyTask));
    upload_sync(d->prefix, prefix.data(), prefix.size() * sizeof(int64_t));
    upload_sync(d->groups, d->host_groups.data(), d->host_groups.size() * sizeof(GemmGroup));
    if (g_multi.size() > 256) g_multi.clear();
    g_multi[key] = d;
    return d;
}
}  // namespace

std::vector<TensorPtr> run_contractions_batched(const std::vector<std::shared_ptr<ContractPlan>>& plans,
                                                const std::vector<const Tensor*>& As,
                                                const std::vector<const Tensor*>& Bs, hipStream_t stream) {
    const int n = (int)plans.size();
    if (n == 0) return {};
    if (n == 1) return {run_contraction(*plans[0], *As[0], *Bs[0], stream)};
    if (n > 4) {   // 3n + 2 buffers must fit the 16-entry pointer table
        std::vector<TensorPtr> out;
        for (int i = 0; i < n; i += 4) {
            const int e = std::min(n, i + 4);
            auto part = run_contractions_batched({plans.begin() + i, plans.begin() + e}, {As.begin() + i, As.begin() + e},
                                                 {Bs.begin() + i, Bs.begin() + e}, stream);
            out.insert(out.end(), part.begin(), part.end());
        }
        return out;
    }
    const Prec prec = plans[0]->prec;
    const bool src64 = As[0]->dtype == SYMTEN_F64;
    for (int i = 0; i < n; ++i) {
        check_device_tensor(*As[i], "contract(A)");
        check_device_tensor(*Bs[i], "contract(B)");
        if (plans[i]->prec != prec || (As[i]->dtype == SYMTEN_F64) != src64)
            fail(SYMTEN_E_INVAL, "batched contractions must share precision and storage type");
    }
    auto d = multi_desc(plans);
    std::vector<TensorPtr> outs(n);
    std::vector<int64_t> sizes(3 * n + 2);
    for (int i = 0; i < n; ++i) {
        outs[i] = std::make_shared<Tensor>(*plans[i]->out_meta);
        outs[i]->meta_only = false;
        outs[i]->buf = device_alloc(std::max<int64_t>(plans[i]->out_elems, 1) * outs[i]->esize());
        sizes[i] = As[i]->elems;
        sizes[n + i] = Bs[i]->elems;
        sizes[2 * n + 2 + i] = plans[i]->out_elems;
    }
    const int pl = panel_planes(prec);
    sizes[2 * n] = pl * d->ap;
    sizes[2 * n + 1] = pl * d->bp;
    if (d->host_groups.empty()) return outs;
    if (d->checked != sizes) {
        validate_tasks(d->host_tasks, sizes, pl);
        validate_groups(d->host_groups, sizes, panel_vw(prec), pl);
        d->checked = sizes;
    }
    const size_t pe = panel_esize(prec) * pl;
    BufferPtr pa = device_alloc(std::max<int64_t>(d->ap, 1) * pe);
    BufferPtr pb = device_alloc(std::max<int64_t>(d->bp, 1) * pe);
    std::vector<void*> ptrs(3 * n + 2);
    for (int i = 0; i < n; ++i) {
        ptrs[i] = As[i]->data();
        ptrs[n + i] = Bs[i]->data();
        ptrs[2 * n + 2 + i] = outs[i]->data();
    }
    ptrs[2 * n] = pa->ptr;
    ptrs[2 * n + 1] = pb->ptr;
    const bool prof = profiling();
    const size_t se = src64 ? 8 : 4;
    profile_launch(copy_kernel_name(src64, prec), 0, 0, prof ? copy_bytes(d->host_tasks, se, pe) : 0, stream, [&] {
        copy_launch_arg((const CopyTask*)d->tasks->ptr, (const int64_t*)d->prefix->ptr, d->ntasks, d->npieces, ptrs,
                        src64, panel_dst_kind(prec), stream);
    });
    auto launch = [&](int cfg) {
        const TileChoice& tc = d->tc;
        BufferPtr ws = tc.ws_bytes[cfg] ? device_alloc(tc.ws_bytes[cfg]) : nullptr;   // split-K partials
        gemm_launch_arg((const TileWork*)tc.tiles[cfg]->ptr, tc.ntiles[cfg], (const GemmGroup*)d->groups->ptr, ptrs,
                        prec, cfg, stream, tc.split(cfg, ws ? ws->ptr : nullptr));
    };
    autotune_gemm(d->tc, d->host_groups, prec, launch, stream);
    const int cfg = d->tc.cfg;
    profile_launch(gemm_kernel_name(prec, cfg), d->info.useful_flops, d->info.gemm_flops,
                   prof ? gemm_bytes(d->host_groups, pe, se) : 0, stream, [&] { launch(cfg); });
    return outs;
}

// ------------------------------------------------------------ double layer
void double_layer_states(const Leg& v, std::vector<int>& ket, std::vector<int>& bra, Leg& fused, int cm) {
    std::vector<int> qs(v.size());
    int o = 0;
    for (size_t s = 0; s < v.q.size(); ++s) {
        for (int i = 0; i < v.d[s]; ++i) qs[o + i] = v.q[s];
        o += v.d[s];
    }
    struct E { int Q, qk, ik, ib; };
    std::vector<E> es;
    for (int ik = 0; ik < v.size(); ++ik)
        for (int ib = 0; ib < v.size(); ++ib) es.push_back({cnorm(qs[ik] - qs[ib], cm), qs[ik], ik, ib});
    std::sort(es.begin(), es.end(), [](const E& x, const E& y) {
        if (x.Q != y.Q) return x.Q < y.Q;
        if (x.qk != y.qk) return x.qk < y.qk;
        if (x.ik != y.ik) return x.ik < y.ik;
        return x.ib < y.ib;
    });
    ket.clear();
    bra.clear();
    fused = Leg();
    fused.dir = v.dir;
    for (auto& e : es) {
        ket.push_back(e.ik);
        bra.push_back(e.ib);
        if (fused.q.empty() || fused.q.back() != e.Q) { fused.q.push_back(e.Q); fused.d.push_back(0); }
        fused.d.back() += 1;
    }
}

TensorPtr double_layer(const Tensor& A, hipStream_t stream, const double* op) {
    if (A.group == SYMTEN_SU2) {
        if (op) fail(SYMTEN_E_UNSUPPORTED, "double_layer: operators take U(1) tensors");
        return double_layer_su2(A, stream);
    }
    check_device_tensor(A, "double_layer");
    if (A.rank() != 5) fail(SYMTEN_E_INVAL, "double_layer: A must have rank 5 (phys, l, u, r, d)");
    const bool f64 = A.dtype == SYMTEN_F64;
    const int np = A.legs[0].size();
    // flux: sum_l dir_l (q_ket - q_bra) = dir_phys (q_s_bra - q_s_ket) for
    // every non-zero op[s_bra][s_ket]
    int flux = 0;
    if (op) {
        if (np > kMaxOpStates) fail(SYMTEN_E_INVAL, "double_layer: operator on more than 8 physical states");
        std::vector<int> qs;
        for (size_t k = 0; k < A.legs[0].q.size(); ++k)
            for (int i = 0; i < A.legs[0].d[k]; ++i) qs.push_back(A.legs[0].q[k]);
        bool any = false;
        for (int sb = 0; sb < np; ++sb)
            for (int sk = 0; sk < np; ++sk) {
                const double v = op[sb * np + sk];
                if (!std::isfinite(v)) fail(SYMTEN_E_INVAL, "double_layer: operator entry not finite");
                if (v == 0.0) continue;
                const int f = cnorm(A.legs[0].dir * (qs[sb] - qs[sk]), charge_mod(A.group));
                if (any && f != flux) fail(SYMTEN_E_SYM, "double_layer: operator does not move the charge by one amount");
                flux = f;
                any = true;
            }
    }
    // fused legs: Q = q_ket - q_bra, states ordered by Q, q_ket, (i_ket, i_bra)
    auto out = std::make_shared<Tensor>();
    out->group = A.group;
    out->flux = flux;
    out->dtype = A.dtype;
    std::vector<std::vector<int>> ket_of(4), bra_of(4);
    for (int l = 0; l < 4; ++l) {
        Leg F;
        double_layer_states(A.legs[l + 1], ket_of[l], bra_of[l], F, charge_mod(A.group));
        out->legs.push_back(F);
    }
    const int64_t total = enumerate_blocks(*out);
    out->elems = total;
    out->meta_only = false;
    out->buf = device_alloc(std::max<int64_t>(total, 1) * out->esize());
    if (total == 0) return out;

    // dense copy of A: [phys][v0][v1][v2][v3]
    std::vector<int> Dv(5);
    for (int l = 0; l < 5; ++l) Dv[l] = A.legs[l].size();
    int64_t dense_n = 1;
    for (int x : Dv) dense_n *= x;
    std::vector<int64_t> dstr = suffix(Dv, 1);
    std::vector<CopyTask> tasks;
    std::vector<std::vector<int>> soff(5);
    for (int l = 0; l < 5; ++l) {
        int o = 0;
        for (int d : A.legs[l].d) { soff[l].push_back(o); o += d; }
    }
    for (auto& b : A.blocks) {
        int64_t doff = 0;
        for (int l = 0; l < 5; ++l) doff += soff[l][A.legs[l].index_of(b.q[l])] * dstr[l];
        std::vector<int64_t> ss(b.stride.begin(), b.stride.end());
        tasks.push_back(make_copy_task(0, b.offset, 1, doff, b.shape, ss, dstr));
    }
    BufferPtr dense = device_alloc(dense_n * out->esize());
    launch_fill_zero(dense->ptr, dense_n * out->esize(), stream);
    std::vector<int64_t> prefix;
    copy_prefix(tasks, prefix);
    BufferPtr dt, dp;
    upload_sync(dt, tasks.data(), tasks.size() * sizeof(CopyTask));
    upload_sync(dp, prefix.data(), prefix.size() * sizeof(int64_t));
    copy_launch_arg((const CopyTask*)dt->ptr, (const int64_t*)dp->ptr, (int)tasks.size(), prefix.back(),
                    {A.data(), dense->ptr}, f64, f64, stream);

    // block tables
    const int nb = (int)out->blocks.size();
    std::vector<int64_t> boff(nb), bstart(nb + 1);
    std::vector<int> bfirst(nb * 4), bshape(nb * 4);
    std::vector<std::vector<int>> foff(4);
    for (int l = 0; l < 4; ++l) {
        int o = 0;
        for (int d : out->legs[l].d) { foff[l].push_back(o); o += d; }
    }
    int64_t acc = 0;
    for (int b = 0; b < nb; ++b) {
        const Block& bl = out->blocks[b];
        boff[b] = bl.offset;
        bstart[b] = acc;
        acc += bl.size;
        for (int l = 0; l < 4; ++l) {
            bfirst[b * 4 + l] = foff[l][out->legs[l].index_of(bl.q[l])];
            bshape[b * 4 + l] = bl.shape[l];
        }
    }
    bstart[nb] = acc;
    std::vector<int> kb;   // ket tables then bra tables, concatenated
    std::vector<int> kb_off(8);
    for (int l = 0; l < 4; ++l) { kb_off[l] = (int)kb.size(); kb.insert(kb.end(), ket_of[l].begin(), ket_of[l].end()); }
    for (int l = 0; l < 4; ++l) { kb_off[4 + l] = (int)kb.size(); kb.insert(kb.end(), bra_of[l].begin(), bra_of[l].end()); }
    BufferPtr d_boff, d_bstart, d_bfirst, d_bshape, d_kb;
    upload_sync(d_boff, boff.data(), boff.size() * 8);
    upload_sync(d_bstart, bstart.data(), bstart.size() * 8);
    upload_sync(d_bfirst, bfirst.data(), bfirst.size() * 4);
    upload_sync(d_bshape, bshape.data(), bshape.size() * 4);
    upload_sync(d_kb, kb.data(), kb.size() * 4);
    DoubleLayerArgs a{};
    a.A_dense = dense->ptr;
    a.nphys = Dv[0];
    for (int l = 0; l < 4; ++l) {
        a.Dv[l] = Dv[l + 1];
        a.ket_of[l] = (const int*)d_kb->ptr + kb_off[l];
        a.bra_of[l] = (const int*)d_kb->ptr + kb_off[4 + l];
    }
    a.blk_off = (const int64_t*)d_boff->ptr;
    a.blk_start = (const int*)d_bfirst->ptr;
    a.blk_shape = (const int*)d_bshape->ptr;
    a.blk_elem_start = (const int64_t*)d_bstart->ptr;
    a.nblocks = nb;
    a.total = total;
    a.out = out->data();
    a.f64 = f64;
    a.has_op = op != nullptr;
    if (op) std::copy(op, op + np * np, a.op);
    launch_double_layer(a, stream);
    // the temporaries go back to the pool; keep ordering by syncing (small)
    HIPCHK(hipStreamSynchronize(stream));
    return out;
}

}  // namespace symten

// ------------------------------------------- unfusing / refusing (ket, bra)
namespace symten {
std::map<int, std::vector<FusedPart>> fused_parts(const Leg& v, int cm) {
    std::map<int, std::vector<FusedPart>> out;
    std::map<int, int> next;
    for (size_t a = 0; a < v.q.size(); ++a)
        for (size_t b = 0; b < v.q.size(); ++b) {
            const int Q = cnorm(v.q[a] - v.q[b], cm);
            FusedPart fp{v.q[a], v.q[b], v.d[a], v.d[b], next[Q]};
            next[Q] += v.d[a] * v.d[b];
            out[Q].push_back(fp);
        }
    return out;
}

namespace {
// Metadata of a tensor with the given legs holding exactly the listed blocks
// (canonical order, contiguous row-major).
TensorPtr tensor_with_blocks(int group, int flux, int dtype, const std::vector<Leg>& legs,
                             std::vector<Block> blocks) {
    auto t = std::make_shared<Tensor>();
    t->group = group;
    t->flux = flux;
    t->dtype = dtype;
    t->legs = legs;
    std::sort(blocks.begin(), blocks.end(), [](const Block& x, const Block& y) { return x.q < y.q; });
    int64_t off = 0;
    for (Block& b : blocks) {
        const int R = (int)b.shape.size();
        b.stride.assign(R, 1);
        for (int l = R - 2; l >= 0; --l) b.stride[l] = b.stride[l + 1] * b.shape[l + 1];
        b.size = 1;
        for (int x : b.shape) b.size *= x;
        b.offset = off;
        off += b.size;
    }
    t->blocks = std::move(blocks);
    t->rebuild_index();
    t->elems = off;
    return t;
}

std::mutex g_gather_mu;
std::map<std::string, std::shared_ptr<GatherPlan>> g_gather_cache;

std::shared_ptr<GatherPlan> make_gather_plan(std::vector<CopyTask>& tasks, const Tensor& src, TensorPtr out,
                                             bool zero) {
    auto g = std::make_shared<GatherPlan>();
    validate_tasks(tasks, {src.elems, out->elems});
    g->ntasks = (int)tasks.size();
    if (!tasks.empty()) {
        std::vector<int64_t> prefix;
        copy_prefix(tasks, prefix);
        upload_sync(g->tasks, tasks.data(), tasks.size() * sizeof(CopyTask));
        upload_sync(g->prefix, prefix.data(), prefix.size() * sizeof(int64_t));
        g->npieces = prefix.back();
    }
    out->buf.reset();
    out->meta_only = true;
    g->meta = out;
    g->zero = zero;
    return g;
}

}  // namespace

TensorPtr run_gather_plan(const GatherPlan& g, const Tensor& src, hipStream_t s) {
    auto out = std::make_shared<Tensor>(*g.meta);
    out->meta_only = false;
    if (g.view) {
        out->buf = src.buf;
        return out;
    }
    out->buf = device_alloc(std::max<int64_t>(out->elems, 1) * out->esize());
    if (g.zero) launch_fill_zero(out->data(), ((std::max<int64_t>(out->elems, 1) * out->esize() + 3) / 4) * 4, s);
    if (g.ntasks > 0) {
        const bool f64 = src.dtype == SYMTEN_F64;
        copy_launch_arg((const CopyTask*)g.tasks->ptr, (const int64_t*)g.prefix->ptr, g.ntasks, g.npieces,
                        {src.data(), out->data()}, f64, f64 ? 1 : 0, s);
    }
    return out;
}

namespace {
std::string leg_key(const Leg& l) {
    std::string k = std::to_string(l.dir) + ":";
    for (size_t i = 0; i < l.q.size(); ++i) k += std::to_string(l.q[i]) + "x" + std::to_string(l.d[i]) + ",";
    return k;
}

std::shared_ptr<GatherPlan> cached(const std::string& key) {
    std::lock_guard<std::mutex> lk(g_gather_mu);
    auto it = g_gather_cache.find(key);
    return it == g_gather_cache.end() ? nullptr : it->second;
}
void remember(const std::string& key, std::shared_ptr<GatherPlan> g) {
    std::lock_guard<std::mutex> lk(g_gather_mu);
    if (g_gather_cache.size() > 512) {
        // launches in flight may still read the task tables
        HIPCHK(hipDeviceSynchronize());
        g_gather_cache.clear();
    }
    g_gather_cache[key] = std::move(g);
}
}  // namespace

TensorPtr unfuse_leg(const Tensor& X, int p, const Leg& v, hipStream_t s) {
    check_device_tensor(X, "unfuse");
    return run_gather_plan(*plan_unfuse(X, p, v), X, s);
}

std::shared_ptr<GatherPlan> plan_unfuse(const Tensor& X, int p, const Leg& v) {
    const std::string key = "u|" + tensor_signature(X) + "|" + std::to_string(p) + "|" + leg_key(v);
    if (auto g = cached(key)) return g;
    const int cm = charge_mod(X.group);
    if (p < 0 || p >= X.rank() || X.rank() + 1 > SYMTEN_MAX_RANK) fail(SYMTEN_E_INVAL, "unfuse: bad leg");
    auto parts = fused_parts(v, cm);
    {
        Leg F;
        for (auto& kv : parts) {
            F.q.push_back(kv.first);
            int n = 0;
            for (auto& fp : kv.second) n += fp.dk * fp.db;
            F.d.push_back(n);
        }
        if (!F.same_sectors(X.legs[p])) fail(SYMTEN_E_LEGS, "unfuse: the leg is not the (ket, bra) fusion of v");
    }
    // Every (ket, bra) part of a fused block is a contiguous run of the fused
    // index, (i_ket, i_bra) row-major: a strided view of the block, so the
    // split tensor shares the source's buffer and nothing is copied.
    auto out = std::make_shared<Tensor>();
    out->group = X.group;
    out->flux = X.flux;
    out->dtype = X.dtype;
    out->legs = X.legs;
    Leg ket = v, bra = v;
    ket.dir = X.legs[p].dir;
    bra.dir = -X.legs[p].dir;
    out->legs[p] = ket;
    out->legs.insert(out->legs.begin() + p + 1, bra);
    for (const Block& b : X.blocks)
        for (const FusedPart& fp : parts.at(b.q[p])) {
            Block n;
            n.q = b.q;
            n.q[p] = fp.qk;
            n.q.insert(n.q.begin() + p + 1, fp.qb);
            n.shape = b.shape;
            n.shape[p] = fp.dk;
            n.shape.insert(n.shape.begin() + p + 1, fp.db);
            n.stride = b.stride;
            n.stride[p] = (int64_t)fp.db * b.stride[p];
            n.stride.insert(n.stride.begin() + p + 1, b.stride[p]);
            n.offset = b.offset + (int64_t)fp.off * b.stride[p];
            n.size = 1;
            for (int x : n.shape) n.size *= x;
            out->blocks.push_back(n);
        }
    std::sort(out->blocks.begin(), out->blocks.end(), [](const Block& x, const Block& y) { return x.q < y.q; });
    out->rebuild_index();
    out->elems = X.elems;
    auto g = std::make_shared<GatherPlan>();
    g->meta = out;
    g->view = true;
    remember(key, g);
    return g;
}

TensorPtr refuse_legs(const Tensor& Z, int pk, int pb, const Leg& F, hipStream_t s) {
    check_device_tensor(Z, "refuse");
    return run_gather_plan(*plan_refuse(Z, pk, pb, F), Z, s);
}

std::shared_ptr<GatherPlan> plan_refuse(const Tensor& Z, int pk, int pb, const Leg& F) {
    const std::string key = "f|" + tensor_signature(Z) + "|" + std::to_string(pk) + "," + std::to_string(pb) + "|" +
                            leg_key(F);
    if (auto g = cached(key)) return g;
    const int cm = charge_mod(Z.group);
    const int R = Z.rank();
    if (pk < 0 || pb < 0 || pk >= R || pb >= R || pk == pb) fail(SYMTEN_E_INVAL, "refuse: bad legs");
    const Leg &lk = Z.legs[pk], &lb = Z.legs[pb];
    if (!lk.same_sectors(lb) || lk.dir != -lb.dir || F.dir != lk.dir)
        fail(SYMTEN_E_LEGS, "refuse: ket and bra legs must be the same sectors, opposite directions");
    auto parts = fused_parts(lk, cm);
    auto newpos = [&](int l) { return l < pb ? l : l - 1; };
    std::vector<Leg> legs;
    for (int l = 0; l < R; ++l)
        if (l != pb) legs.push_back(l == pk ? F : Z.legs[l]);
    std::map<std::vector<int>, Block> targets;
    struct Src { const Block* b; std::vector<int> key; int off, db; };
    std::vector<Src> srcs;
    for (const Block& b : Z.blocks) {
        const int Q = cnorm(b.q[pk] - b.q[pb], cm);
        int off = -1, db = 0;
        for (const FusedPart& fp : parts.at(Q))
            if (fp.qk == b.q[pk]) { off = fp.off; db = fp.db; }
        if (off < 0 || F.dim_of(Q) == 0) fail(SYMTEN_E_LEGS, "refuse: fused sector missing");
        Block t;
        for (int l = 0; l < R; ++l) {
            if (l == pb) continue;
            t.q.push_back(l == pk ? Q : b.q[l]);
            t.shape.push_back(l == pk ? F.dim_of(Q) : b.shape[l]);
        }
        targets[t.q] = t;
        srcs.push_back({&b, t.q, off, db});
    }
    std::vector<Block> tb;
    for (auto& kv : targets) tb.push_back(kv.second);
    TensorPtr out = tensor_with_blocks(Z.group, Z.flux, Z.dtype, legs, tb);
    std::vector<CopyTask> tasks;
    for (const Src& sr : srcs) {
        const Block& d = out->blocks[out->index.at(sr.key)];
        std::vector<int64_t> ds(R);
        const int pkn = newpos(pk);
        for (int l = 0; l < R; ++l) {
            if (l == pk) ds[l] = (int64_t)sr.db * d.stride[pkn];
            else if (l == pb) ds[l] = d.stride[pkn];
            else ds[l] = d.stride[newpos(l)];
        }
        std::vector<int64_t> ss(sr.b->stride.begin(), sr.b->stride.end());
        tasks.push_back(make_copy_task(0, sr.b->offset, 1, d.offset + (int64_t)sr.off * d.stride[pkn], sr.b->shape, ss,
                                       ds));
    }
    auto g = make_gather_plan(tasks, Z, out, true);
    remember(key, g);
    return g;
}
}  // namespace symten
