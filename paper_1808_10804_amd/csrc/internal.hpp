// Internal data structures of libsymten: tensor metadata, contraction plans,
// device work descriptors and the kernel launch interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <map>
#include <mutex>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/symten.h"

namespace symten {

// ---------------------------------------------------------------- errors ---
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define HIPCHK(x) ::symten::hip_check((x), #x)

// ------------------------------------------------------------------ legs ---
struct Leg {
    int dir = 1;                 // +1 in, -1 out
    std::vector<int> q;          // charges, ascending
    std::vector<int> d;          // dims (all > 0)
    int size() const { int s = 0; for (int x : d) s += x; return s; }
    int index_of(int charge) const {
        for (size_t i = 0; i < q.size(); ++i) if (q[i] == charge) return (int)i;
        return -1;
    }
    int dim_of(int charge) const { int i = index_of(charge); return i < 0 ? 0 : d[i]; }
    bool same_sectors(const Leg& o) const { return q == o.q && d == o.d; }
};

// ----------------------------------------------------------------- blocks ---
struct Block {
    std::vector<int> q;          // charge per leg (SU(2): doubled spin 2j)
    std::vector<int> tree;       // SU(2) coupling-tree labels (empty for U(1))
    std::vector<int> shape;      // dims per leg
    std::vector<int64_t> stride; // element strides per leg
    int64_t offset = 0;          // element offset into the tensor buffer
    int64_t size = 0;
};

// Stream of the library call running on this thread (entry points that take
// a stream set it for their duration; host threads of the library set their
// own).  Outside a call it is unset.
struct StreamScope {
    hipStream_t prev;
    bool prev_set;
    explicit StreamScope(hipStream_t s);
    ~StreamScope();
};
bool call_stream_set();
hipStream_t call_stream();

// Caching device allocator (size-bucketed free lists).  A released block
// records an event on the stream that released it: the stream of the call
// running on the releasing thread, else the stream the block was allocated
// on.  Handing the block to a call on another stream makes that stream wait
// for the event, so work queued on two streams never shares a block.
struct DeviceBuffer;
using BufferPtr = std::shared_ptr<DeviceBuffer>;
BufferPtr device_alloc(size_t bytes);
struct DeviceBuffer {
    void* ptr = nullptr;
    size_t bytes = 0;
    size_t cap = 0;
    hipStream_t stream = nullptr;   // stream of the call that allocated it
    // set when a caller-registered allocator made the buffer
    void (*user_free)(void* ptr, size_t bytes, void* ctx) = nullptr;
    void* user_ctx = nullptr;
    uint64_t user_gen = 0;  // registration that made it; a later one leaks it
    ~DeviceBuffer();
};
// Caller-registered device allocator (null fns: the library's own pool).
void set_user_allocator(void* (*alloc)(size_t, void*), void (*free_fn)(void*, size_t, void*), void* ctx);

// A tensor's layout signature, computed on first use and kept: copies start
// without one (they are usually edited before use) and rebuild_index(), the
// last step of every layout edit, drops it.
struct SignatureMemo {
    std::mutex mu;
    std::string sig;
    bool valid = false;
    SignatureMemo() = default;
    SignatureMemo(const SignatureMemo&) {}
    SignatureMemo& operator=(const SignatureMemo&) {
        std::lock_guard<std::mutex> lk(mu);
        valid = false;
        sig.clear();
        return *this;
    }
    void reset() {
        std::lock_guard<std::mutex> lk(mu);
        valid = false;
        sig.clear();
    }
};

struct Tensor {
    int group = SYMTEN_U1;
    int flux = 0;
    int dtype = SYMTEN_F32;
    std::vector<Leg> legs;
    std::vector<Block> blocks;               // canonical (lexicographic) order
    std::map<std::vector<int>, int> index;   // labels (charges, then tree) -> block index
    BufferPtr buf;                           // null for metadata-only handles
    int64_t elems = 0;                       // buffer size in elements
    bool meta_only = true;
    mutable SignatureMemo memo;              // tensor_signature's result

    int rank() const { return (int)legs.size(); }
    int64_t nnz() const { int64_t s = 0; for (auto& b : blocks) s += b.size; return s; }
    size_t esize() const { return dtype == SYMTEN_F64 ? 8 : 4; }
    void* data() const { return buf ? buf->ptr : nullptr; }
    void rebuild_index();
};
using TensorPtr = std::shared_ptr<Tensor>;

// Abelian groups: U(1) charges are integers, Z2 charges parities 0, 1 with
// every sum taken mod 2.  charge_mod is 0 for U(1), 2 for Z2; cnorm brings a
// sum of charges back to its label.
inline int charge_mod(int group) { return group == SYMTEN_Z2 ? 2 : 0; }
inline int cnorm(long q, int m) { return m ? (int)(((q % m) + m) % m) : (int)q; }
inline bool abelian(int group) { return group == SYMTEN_U1 || group == SYMTEN_Z2; }

// Allowed blocks of the given legs and flux, canonical order, contiguous
// row-major layout; returns total element count.
int64_t enumerate_blocks(Tensor& t);
// SU(2): one block per (spin per leg, coupling tree), lexicographic.
int64_t enumerate_blocks_su2(Tensor& t);
// Clebsch-Gordan coefficient <j1 m1; j2 m2 | J M>, all arguments doubled.
double cg_coeff(int tj1, int tm1, int tj2, int tm2, int tJ, int tM);

// ------------------------------------------------------------- device ops ---
// Strided copy task: iterate a multi-index over dims (last fastest);
// dst[dst_off + sum i*dstride] = src[src_off + sum i*sstride] (or 0 when
// src_buf < 0).  Buffers are named by index into a pointer table.
// A task may also sum several equally strided sources of the same buffer:
// dst = scale * src[src_off + i] + sum_t xscale[t] * src[xsrc_off[t] + i]
// (SU(2) operands: blocks that differ only in their coupling tree are
// combined with their recoupling scalars before the product).
constexpr int kMaxCopyRank = 8;
constexpr int kMaxExtraSrc = 7;
struct CopyTask {
    int64_t src_off, dst_off;
    int64_t sstride[kMaxCopyRank];
    int64_t dstride[kMaxCopyRank];
    int dims[kMaxCopyRank];
    int rank;
    int src_buf, dst_buf;
    int count;          // product of dims (< 2^31)
    double scale;       // multiplies the copied value (SU(2) recoupling scalar)
    int64_t lo_off;     // split panels: plane p starts p * lo_off elements after the hi plane
    int nextra;         // number of extra sources (0 .. kMaxExtraSrc)
    int nchunks;        // chunks of the task (copy_task_chunks)
    int64_t xsrc_off[kMaxExtraSrc];
    double xscale[kMaxExtraSrc];
    // transposing copy (the destination's unit-stride dim is not the
    // source's): tiles of (1 << lg_out) x (1024 >> lg_out) elements staged
    // through LDS, read along dim tr_in, written along dim tr_out; -1: direct
    int tr_in, tr_out, lg_out, pad2_;
};
// chunks of a copy task: 1024 elements, or one LDS tile of 1024
int64_t copy_task_chunks(const CopyTask& t);
// A workgroup of the gather takes up to kCopyGroup consecutive chunks of one
// task (a piece); the prefix sums handed to the copy launches count pieces.
constexpr int kCopyGroup = 4;

struct GemmGroup {
    int64_t a_off, b_off, c_off;   // element offsets into their buffers
    int M, N, K;
    int lda, ldb, ldc;             // A: [M][lda] (K contiguous); B: [N][ldb]; C: [M][ldc]
    int a_buf, b_buf, c_buf;
    int tiles_n;                   // tiles along N (for tile decoding)
    int scatter;                   // 0: C written at c_off; 1: scatter epilogue (below)
    int64_t a_lo, b_lo;            // split panels: plane p starts p * a_lo (p * b_lo) elements in
    // Scatter epilogue (bf16 kernels): element (i, j) goes, split into the
    // kernel's bf16 planes (plane p at p * c_lo), to c_buf at
    //   d0 + sum_l rows[i].idx[l] * sr[l] + sum_l cols[j].idx[l] * sc[l]
    // with (d0, sr, sc) the entry (rows[i].blk, cols[j].blk) of the block
    // table (d0 < 0: the element is dropped).  The tables are int32 records
    // in buffer s_buf: rows {blk, idx[3]}, cols {blk, idx[3]}, blocks
    // {d0, sr[3], sc[3], pad}, starting at s_rows, s_cols, s_blocks (in
    // ints); the block table has s_ncb entries per row block.
    int s_buf, s_ncb;
    int64_t s_rows, s_cols, s_blocks, c_lo;
};
constexpr int kScatterLegs = 3;   // row (column) legs a scatter epilogue decodes


// One work item of a grouped-GEMM launch: output tile (tm, tn) of a group,
// over the K range [k0, k1).  slot < 0: the item writes its C tile; else the
// item is one part of a split K and writes its partial tile to slot `slot`
// of the launch's workspace.  group < 0: padding (no work).
struct TileWork {
    int group, tm, tn;
    int k0, k1;
    int slot;
    int pad0, pad1;
};
// An output tile computed as nparts K parts: their partial tiles, workspace
// slots slot0 .. slot0 + nparts - 1, are added in that order into C.
struct SplitOut {
    int group, tm, tn, slot0, nparts, pad;
};
// The work list of one launch with a tile configuration.
struct TilePlan {
    std::vector<TileWork> tiles;
    std::vector<SplitOut> splits;
    int64_t partial_tiles = 0;     // workspace slots
};
// Workspace of a launch: the persistent grid's per-XCD queue counters
// (kSplitQueueBytes), then the split-K partial tiles.
constexpr int64_t kSplitQueueBytes = 256;
struct SplitK {
    const SplitOut* splits = nullptr;
    int nsplits = 0;
    void* ws = nullptr;            // queue counters, then partial tiles BM x BN (FP64 or FP32 by precision)
};

// Pointer table handed to the kernels (device addresses).
constexpr int kMaxBufs = 512;

// Element type of a panel / buffer in a GEMM launch.
enum class Prec { F64 = 0, F32 = 1, BF16 = 2, BF16X3 = 3, BF16X6 = 4 };

// Panel element type per precision: FP64 -> double, FP32 -> float,
// BF16 -> one bf16 plane, BF16X3 -> bf16 hi and lo planes, BF16X6 -> bf16
// hi, mid and lo planes.  The planes of a panel buffer are consecutive
// copies of its layout, plane p starting p * (plane stride) elements in.
inline size_t panel_esize(Prec p) { return p == Prec::F64 ? 8 : (p == Prec::F32 ? 4 : 2); }
inline int panel_planes(Prec p) { return p == Prec::BF16X3 ? 2 : (p == Prec::BF16X6 ? 3 : 1); }
inline int panel_vw(Prec p) { return p == Prec::F64 ? 2 : (p == Prec::F32 ? 4 : 8); }   // 16-byte vectors

// Gather launch over a task list already on the device (at most 16 buffers).
// dst_kind: 0 float, 1 double, 2 bf16, 3 bf16 hi/lo split, 4 accumulate
// (dst += scale * src, source type), 5 bf16 hi/mid/lo split.
void copy_launch_arg(const CopyTask* d_tasks, const int64_t* d_prefix, int ntasks, int64_t npieces,
                     const std::vector<void*>& ptrs, bool src_f64, int dst_kind, hipStream_t s);

void launch_cast(const void* src, bool src_f64, void* dst, bool dst_f64, int64_t n, hipStream_t s);
void launch_fill_zero(void* dst, int64_t bytes, hipStream_t s);
// table[idx] = p on the device, ordered on stream s.
void launch_set_pointer(void** table, int idx, void* p, hipStream_t s);
// FP64 sum of squares of n elements into *out (device double), then scale.
void launch_sumsq(const void* x, bool f64, int64_t n, double* out, hipStream_t s);
void launch_scale_by_inv_sqrt(void* x, bool f64, int64_t n, const double* sumsq, hipStream_t s);

// Double layer.  Fused-leg tables are device int arrays.
constexpr int kMaxOpStates = 8;   // physical states of a one-site operator
struct DoubleLayerArgs {
    const void* A_dense;   // [phys][D0][D1][D2][D3] dense copy of A (same dtype)
    int nphys, Dv[4];
    const int* ket_of[4];  // fused state -> ket state
    const int* bra_of[4];
    const int64_t* blk_off;   // per output block offset
    const int* blk_start;     // per output block first fused state per leg [nb*4]
    const int* blk_shape;     // [nb*4]
    const int64_t* blk_elem_start; // prefix of block sizes [nb+1]
    int nblocks;
    int64_t total;
    void* out;
    bool f64;
    // optional one-site operator between the layers: out = sum over
    // (s_bra, s_ket) of op[s_bra * nphys + s_ket] A[s_ket] (ket) A[s_bra] (bra)
    bool has_op;
    double op[kMaxOpStates * kMaxOpStates];
};
void launch_double_layer(const DoubleLayerArgs& a, hipStream_t s);
// scatter of a contiguous-block tensor into a dense array
void launch_sign_fix_rows(double* Pt, int ldPt, int rows, int n, double* P, int ldP, hipStream_t s);
// FP64 symmetric eigensolver of the projector stage (eig.hip).  Phase one
// enqueues the tridiagonalisations and all eigenvalues (w, ascending);
// phase two, once the caller has the eigenvalues on the host, the
// eigenvectors of the kv[i] largest into Z[i] (n x kv, column-major, column
// j for the (j+1)-th largest).  The work object keeps the buffers the
// phases share.
struct EighProblem {
    int n = 0, lda = 0;
    const double* A = nullptr;   // n x n, column-major, both triangles
    double* w = nullptr;         // n eigenvalues, ascending
    int* status = nullptr;       // optional, zeroed by the caller: set to 1 if
                                 // the tridiagonalisation's barrier gave up
};
struct EighWork;
bool eigh_fits(int n);
int eigh_problems(const EighWork& wk);
int eigh_max_order();
std::shared_ptr<EighWork> eigh_values(const std::vector<EighProblem>& probs, hipStream_t s);
// synchronises s; fails if a tridiagonalisation's workgroups did not meet
void eigh_status(const EighWork& wk, hipStream_t s);
void eigh_vectors(EighWork& wk, const std::vector<int>& kv, const std::vector<double*>& Z,
                  const std::vector<const double*>& w_host, hipStream_t s);

// -------------------------------------------------------------- contraction --
struct GroupPlan {
    int key;                      // contracted charge as seen from A
    int M, N, K, lda;
    int64_t a_off, b_off, c_off;  // into A panel ws, B panel ws, output buffer
    std::vector<std::vector<int>> rows;   // alpha tuples (charges), in order
    std::vector<std::vector<int>> cols;   // beta tuples
    std::vector<int> row_off, col_off;
};

// Where the elements of one block of A land in the A panels: element
// (idx_0 .. idx_{R-1}) of block `block` (legs in A's order) goes to panel
// offset dst_off + sum_l idx_l * dstride[l].  One entry per A block that a
// U(1) or Z2 plan gathers (with scale 1 and one source).
struct PanelMap {
    int block;
    int64_t dst_off;
    std::vector<int64_t> dstride;
};

struct ContractPlan {
    TensorPtr out_meta;                   // metadata of the output (no buffer)
    std::vector<GroupPlan> groups;
    std::vector<CopyTask> copies;         // bufs: 0 = A data, 1 = B data, 2 = A panels, 3 = B panels
    std::vector<PanelMap> a_maps;         // the A-side copies of `copies` as block maps (abelian plans)
    std::vector<int> conA, conB;          // contracted legs (abelian plans)
    int64_t a_panel_elems = 0, b_panel_elems = 0, out_elems = 0;
    symten_plan_stats info{};
    Prec prec = Prec::F32;
    bool panel_f64 = false;
    mutable std::shared_ptr<void> dev;    // device copies of the descriptors
};

// Strided copy task over dims (last fastest); simplified (unit dims dropped,
// contiguous dims merged).  src_buf < 0 writes zeros.
CopyTask make_copy_task(int src_buf, int64_t src_off, int dst_buf, int64_t dst_off, const std::vector<int>& dims,
                        const std::vector<int64_t>& sstr, const std::vector<int64_t>& dstr, double scale = 1.0);

// Expansion of an SU(2) tensor into the U(1) tensor of its S^z components
// (charges 2m; within a charge, states by spin then multiplet index).
// The SU(2) double layer of A with `op` (null: identity) between the layers
// on the physical S^z states, left as a U(1) tensor in the S^z basis of the
// fused multiplets (the basis su2_to_u1 gives an environment's D^2 legs).
TensorPtr double_layer_su2_sz(const Tensor& A, const double* op, hipStream_t stream);
TensorPtr su2_to_u1(const Tensor& in, hipStream_t stream);

// SU(2) part of plan_contraction, called after the leg checks.
std::shared_ptr<ContractPlan> plan_contraction_su2(const Tensor& A, const Tensor& B, const std::vector<int>& conA,
                                                   const std::vector<int>& conB, const std::vector<int>& freeA,
                                                   const std::vector<int>& freeB, const std::vector<int>& perm,
                                                   Prec p);

// Build the plan (host only).  Throws Error on invalid input.
std::shared_ptr<ContractPlan> plan_contraction(const Tensor& A, const Tensor& B, int ncon,
                                               const int* legsA, const int* legsB,
                                               const int* out_perm, int prec);

// The plan's GEMM groups launched with a tile list (at most 16 buffers):
// a persistent grid that holds as many workgroups as the chip runs at once
// walks the list; split-K parts are added afterwards in a fixed order.
void gemm_launch_arg(const TileWork* d_tiles, int ntiles, const GemmGroup* d_groups,
                     const std::vector<void*>& ptrs, Prec prec, int cfg, hipStream_t s, const SplitK& sk = {});
// scatter: every group of the launch has the scatter epilogue (bf16 precisions)
void gemm_launch_dev(const TileWork* d_tiles, int ntiles, const GemmGroup* d_groups, void* const* d_ptrs,
                     Prec prec, int cfg, hipStream_t s, const SplitK& sk = {}, bool scatter = false);
// Workgroups of a tile configuration that the chip holds at once (occupancy
// times compute units).
int gemm_capacity(Prec p, int cfg);
// Lists longer than kPersistentFactor times the capacity run on a persistent
// grid that takes entries from per-XCD queues.
constexpr int kPersistentFactor = 4;
bool gemm_persistent(int ntiles, int capacity);
// Tile configuration used without the autotuner.
int choose_tile_cfg(const ContractPlan& p);
// The plan of a contraction from the library's plan cache.
std::shared_ptr<ContractPlan> cached_plan(const Tensor& A, const Tensor& B, int ncon, const int* la, const int* lb,
                                          const int* perm, int prec);
// Contraction of a plan into the caller's tensor `out` (contiguous blocks,
// the plan's legs) through the library's fixed device work area: no device
// allocation.
void contract_noalloc(Tensor& out, const Tensor& A, const Tensor& B, const std::shared_ptr<ContractPlan>& plan,
                      hipStream_t s);

// Sector matching of a contraction on the device (see symten_match_blocks).
void match_blocks(const Tensor& A, const Tensor& B, int ncon, const int* legsA, const int* legsB,
                  symten_pair* pairs, int64_t pair_cap, int* out_labels, int64_t out_cap, int64_t* counts,
                  hipStream_t s);

// Execute a plan: allocates the output buffer, gathers panels, runs the GEMMs.
TensorPtr run_contraction(const ContractPlan& p, const Tensor& A, const Tensor& B,
                          hipStream_t stream);

// Execute many plans with one gather launch and one GEMM launch.
std::vector<TensorPtr> run_contractions_batched(
    const std::vector<std::shared_ptr<ContractPlan>>& plans, const std::vector<const Tensor*>& As,
    const std::vector<const Tensor*>& Bs, hipStream_t stream);

// plan / descriptor helpers shared by the launch paths
void upload_sync(BufferPtr& buf, const void* host, size_t bytes);
// Work list of a launch; with allow_split, tiles of a launch that would not
// fill the chip are split along K (see the definition).
void build_tiles(const std::vector<GemmGroup>& groups, Prec prec, int cfg, TilePlan& tp, bool allow_split);
void copy_prefix(const std::vector<CopyTask>& tasks, std::vector<int64_t>& prefix);
// planes: panel planes a split destination writes (plane p at p * lo_off)
void validate_tasks(const std::vector<CopyTask>& tasks, const std::vector<int64_t>& buf_elems, int planes = 1);
// Scatter tables (appended to `tab`) for the groups of plan p, whose products
// are the A operand of plan q: each product goes to the position of q's A
// panels (offset by a_base) that q's gather would copy it to.  Sets the
// table fields of groups[0 .. p.groups.size()) (the launch's copies of p's
// groups, in order); the caller sets s_buf, c_buf and c_lo.  Returns the
// number of products that reach a panel.
int64_t append_scatter_tables(const ContractPlan& p, const Tensor& A, const Tensor& B, const ContractPlan& q,
                              int64_t a_base, GemmGroup* groups, std::vector<int>& tab);
// The scatter groups' tables (int32 records in `tab`) and every destination
// they reach, against a destination of dst_elems elements with `planes` planes.
void validate_scatter(const std::vector<GemmGroup>& groups, const std::vector<int>& tab, int64_t dst_elems,
                      int planes);
void validate_groups(const std::vector<GemmGroup>& groups, const std::vector<int64_t>& buf_elems, int vw,
                     int planes = 1);

// op (may be null): nphys x nphys row-major over A's physical states,
// op[s_bra][s_ket]; every non-zero entry must move the charge by the same
// amount (the result's flux follows from it).
TensorPtr double_layer(const Tensor& A, hipStream_t stream, const double* op = nullptr);
// SU(2) double layer (S^z components, U(1) double layer, per-leg change to
// the fused multiplet basis, reduction).
TensorPtr double_layer_su2(const Tensor& A, hipStream_t stream);
// Fused (ket, bra) states of a U(1) double-layer leg: charge q_ket - q_bra,
// ordered by that charge, then q_ket, then (i_ket, i_bra); ket/bra are state
// indices of the leg (charge-major order).
void double_layer_states(const Leg& v, std::vector<int>& ket, std::vector<int>& bra, Leg& fused, int cm = 0);
// The (ket, bra) parts of each sector Q of a double-layer leg fused from v:
// ket charge ascending, each a contiguous run of dk * db fused states.
struct FusedPart { int qk, qb, dk, db, off; };
std::map<int, std::vector<FusedPart>> fused_parts(const Leg& v, int cm);
// Leg p of X (a double-layer leg fused from v) split into a ket leg (v, the
// leg's direction) at p and a bra leg (v, reversed) at p + 1; the result's
// blocks are strided views of X's buffer.
TensorPtr unfuse_leg(const Tensor& X, int p, const Leg& v, hipStream_t s);
// The ket leg pk and bra leg pb of Z fused into F (the double-layer fusion of
// the ket leg) at position pk, pb removed; one gather into a zeroed buffer.
TensorPtr refuse_legs(const Tensor& Z, int pk, int pb, const Leg& F, hipStream_t s);
// The two as reusable plans (output layout + device task table, cached by
// source layout and arguments) and their execution into a new tensor.
struct GatherPlan {
    TensorPtr meta;            // output tensor without storage
    BufferPtr tasks, prefix;   // device copy tasks (buffer 0: source, 1: output)
    int ntasks = 0;
    int64_t npieces = 0;
    bool zero = false;         // output parts not covered by a task are zero
    bool view = false;         // the output's blocks are views of the source's buffer
};
std::shared_ptr<GatherPlan> plan_unfuse(const Tensor& X, int p, const Leg& v);
std::shared_ptr<GatherPlan> plan_refuse(const Tensor& Z, int pk, int pb, const Leg& F);
TensorPtr run_gather_plan(const GatherPlan& g, const Tensor& src, hipStream_t s);
// SU(2) tensor with legs `legs` from the U(1) tensor of its S^z components
// (the inverse of su2_to_u1 on invariant tensors): projection of every block
// onto its basis tensor.
TensorPtr u1_to_su2(const Tensor& U, const std::vector<Leg>& legs, hipStream_t stream);
// SU(2) tensor with its legs permuted (new leg j = old leg perm[j]) and the
// legs `flip` (new positions) reversed, through the S^z components: a
// reversed leg maps the state (j, m) to (j, -m) with the phase (-1)^(j-m).
// Reversing both ends of a bond leaves a network unchanged; reversing a leg
// twice multiplies its half-integer spins by -1.
TensorPtr su2_permute_flip(const Tensor& X, const std::vector<int>& perm, const std::vector<int>& flip,
                           hipStream_t s);
// X with the blocks of half-integer spin on `leg` multiplied by -1.
TensorPtr su2_sign_half_integer(const Tensor& X, int leg, hipStream_t s);

// GEMM tile shapes and the autotuner that picks one per launch
constexpr int kNumTileCfg = 8;
int gemm_tile_bm(Prec p, int cfg);
int gemm_tile_bn(Prec p, int cfg);
int gemm_tile_bk(Prec p, int cfg);
bool gemm_tile_ok(Prec p, int cfg);
struct TileChoice {
    int cfg = -1;                          // chosen configuration (-1: not tuned)
    BufferPtr tiles[kNumTileCfg];          // device work lists per configuration
    BufferPtr splits[kNumTileCfg];         // device split-K output lists
    int ntiles[kNumTileCfg] = {};
    int nsplits[kNumTileCfg] = {};
    int64_t ws_bytes[kNumTileCfg] = {};    // split-K workspace a launch needs
    float ms[kNumTileCfg] = {};
    // split-K arguments of configuration c with workspace ws
    SplitK split(int c, void* ws) const {
        return SplitK{nsplits[c] ? (const SplitOut*)splits[c]->ptr : nullptr, nsplits[c], ws};
    }
};
// Picks the tile configuration for this set of GEMM groups: a cached
// decision for the same shapes, else each available configuration is timed
// once with HIP events through `launch(cfg)` (idempotent: C = A B is
// rewritten), after ensure_tiles(cfg).  Must not be called while the stream
// is being captured.
void autotune_gemm(TileChoice& tc, const std::vector<GemmGroup>& groups, Prec prec,
                   const std::function<void(int cfg)>& launch, hipStream_t s);
void ensure_tiles(TileChoice& tc, const std::vector<GemmGroup>& groups, Prec prec, int cfg);

// kernel timing (events around launches while enabled)
bool profiling();
void profile_launch(const std::string& name, int64_t uf, int64_t gf, int64_t bytes, hipStream_t s,
                    const std::function<void()>& launch);
void profile_begin();
std::vector<symten_kernel_stat> profile_end();
std::string gemm_kernel_name(Prec p, int cfg, bool scatter = false);
std::string copy_kernel_name(bool src64, Prec p);
int panel_dst_kind(Prec p);
int64_t copy_bytes(const std::vector<CopyTask>& tasks, size_t se, size_t de);
int64_t gemm_bytes(const std::vector<GemmGroup>& gs, size_t pe, size_t oe);

// helpers
std::string tensor_signature(const Tensor& t);
void check_device_tensor(const Tensor& t, const char* what);

}  // namespace symten
