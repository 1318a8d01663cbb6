// Block-sparse contraction into a caller's tensor with no device allocation,
// for callers that cannot allocate (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// Every piece of device memory the contraction needs beyond its inputs and
// its output -- the copy-task and GEMM descriptors, the tile list, the
// gathered A and B panels and the charge-sector products -- lives in one
// file-scope device array of fixed size.  Each GPU holds its own copy of the
// array for the life of the process; its device address is looked up once
// per device with hipGetSymbolAddress and only that address is handed to the
// kernels and copies (the array's name is a host-side stand-in in host code).
// Calls on one GPU share the array, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace symten {

static __device__ __align__(256) unsigned char scratch[SYMTEN_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up on the first
// call on the device (with that device current).
void* scratch_address() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(SYMTEN_E_CAPACITY, "contract_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(SYMTEN_E_HIP, "contract_noalloc: no device address for the work area");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// Host image of the descriptor part of the work area, laid out as it will
// be on the device.
struct Blob {
    std::vector<unsigned char> bytes;
    int64_t put(const void* src, size_t n) {
        const int64_t off = align256((int64_t)bytes.size());
        bytes.resize(off + n);
        if (n) std::memcpy(bytes.data() + off, src, n);
        return off;
    }
};

bool same_legs(const Tensor& x, const Tensor& y) {
    if (x.rank() != y.rank()) return false;
    for (int l = 0; l < x.rank(); ++l)
        if (x.legs[l].dir != y.legs[l].dir || !x.legs[l].same_sectors(y.legs[l])) return false;
    return true;
}
}  // namespace

void contract_noalloc(Tensor& out, const Tensor& A, const Tensor& B, const std::shared_ptr<ContractPlan>& plan,
                      hipStream_t s) {
    const ContractPlan& p = *plan;
    const Tensor& meta = *p.out_meta;
    check_device_tensor(A, "contract_noalloc(A)");
    check_device_tensor(B, "contract_noalloc(B)");
    check_device_tensor(out, "contract_noalloc(out)");
    if (out.group != meta.group || out.flux != meta.flux || out.dtype != meta.dtype || !same_legs(out, meta))
        fail(SYMTEN_E_INVAL, "contract_noalloc: out must have the contraction's legs, flux and storage type");
    const int R = out.rank();
    const size_t oe = out.esize();
    // out's blocks must be contiguous row-major (as symten_create makes them)
    for (const Block& b : out.blocks) {
        int64_t st = 1;
        for (int l = R - 1; l >= 0; --l) {
            if (b.shape[l] > 1 && b.stride[l] != st) fail(SYMTEN_E_INVAL, "contract_noalloc: out blocks must be contiguous");
            st *= b.shape[l];
        }
    }
    // ---- descriptors (host) ------------------------------------------------
    const int pl = panel_planes(p.prec);
    const size_t pe = panel_esize(p.prec);
    std::vector<GemmGroup> groups;
    for (auto& g : p.groups) {
        GemmGroup x{};
        x.a_off = g.a_off;
        x.b_off = g.b_off;
        x.c_off = g.c_off;
        x.M = g.M;
        x.N = g.N;
        x.K = g.K;
        x.lda = x.ldb = g.lda;
        x.ldc = g.N;
        x.a_buf = 0;
        x.b_buf = 1;
        x.c_buf = 2;
        if (pl > 1) {
            x.a_lo = p.a_panel_elems;
            x.b_lo = p.b_panel_elems;
        }
        groups.push_back(x);
    }
    const int cfg = choose_tile_cfg(p);
    TilePlan tp;                 // no split K: no workspace beyond the panels
    if (!groups.empty()) build_tiles(groups, p.prec, cfg, tp, false);
    const std::vector<TileWork>& tiles = tp.tiles;
    std::vector<int64_t> prefix;
    copy_prefix(p.copies, prefix);
    // the charge-sector products (buffer 0) scattered into out's blocks (buffer 1)
    std::vector<CopyTask> scatter;
    for (const Block& b : meta.blocks) {
        auto it = out.index.find(b.q);
        if (it == out.index.end()) fail(SYMTEN_E_INVAL, "contract_noalloc: out lacks a block of the contraction");
        const Block& d = out.blocks[it->second];
        scatter.push_back(make_copy_task(0, b.offset, 1, d.offset, b.shape, b.stride, d.stride));
    }
    std::vector<int64_t> sprefix;
    copy_prefix(scatter, sprefix);
    validate_tasks(p.copies, {A.elems, B.elems, pl * p.a_panel_elems, pl * p.b_panel_elems}, pl);
    validate_groups(groups, {pl * p.a_panel_elems, pl * p.b_panel_elems, std::max<int64_t>(p.out_elems, 1)},
                    panel_vw(p.prec), pl);
    validate_tasks(scatter, {std::max<int64_t>(p.out_elems, 1), out.elems});

    Blob blob;
    const int64_t o_tasks = blob.put(p.copies.data(), p.copies.size() * sizeof(CopyTask));
    const int64_t o_prefix = blob.put(prefix.data(), prefix.size() * sizeof(int64_t));
    const int64_t o_groups = blob.put(groups.data(), groups.size() * sizeof(GemmGroup));
    const int64_t o_tiles = blob.put(tiles.data(), tiles.size() * sizeof(TileWork));
    const int64_t o_scat = blob.put(scatter.data(), scatter.size() * sizeof(CopyTask));
    const int64_t o_sprefix = blob.put(sprefix.data(), sprefix.size() * sizeof(int64_t));
    const int64_t o_queue = align256((int64_t)blob.bytes.size());   // the persistent grid's counters
    const int64_t o_pa = align256(o_queue + kSplitQueueBytes);
    const int64_t o_pb = align256(o_pa + (int64_t)pe * pl * p.a_panel_elems);
    const int64_t o_c = align256(o_pb + (int64_t)pe * pl * p.b_panel_elems);
    const int64_t need = o_c + (int64_t)oe * p.out_elems;
    if (need > (int64_t)SYMTEN_NOALLOC_SCRATCH_BYTES)
        fail(SYMTEN_E_CAPACITY, "contract_noalloc: the contraction needs " + std::to_string(need) +
                                    " bytes of work area, more than the " +
                                    std::to_string((int64_t)SYMTEN_NOALLOC_SCRATCH_BYTES) + " available");

    // ---- device work ---------------------------------------------------------
    unsigned char* w = (unsigned char*)scratch_address();
    // the caller's blocks that no pair reaches are zero
    launch_fill_zero(out.data(), (std::max<int64_t>(out.elems, 1) * (int64_t)oe + 3) / 4 * 4, s);
    if (groups.empty()) return;
    // descriptors: pageable host memory, consumed by the runtime before the
    // copy call returns
    HIPCHK(hipMemcpyAsync(w, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice, s));
    const bool src64 = A.dtype == SYMTEN_F64;
    copy_launch_arg((const CopyTask*)(w + o_tasks), (const int64_t*)(w + o_prefix), (int)p.copies.size(),
                    prefix.back(), {A.data(), B.data(), w + o_pa, w + o_pb}, src64, panel_dst_kind(p.prec), s);
    gemm_launch_arg((const TileWork*)(w + o_tiles), (int)tiles.size(), (const GemmGroup*)(w + o_groups),
                    {w + o_pa, w + o_pb, w + o_c}, p.prec, cfg, s, SplitK{nullptr, 0, w + o_queue});
    copy_launch_arg((const CopyTask*)(w + o_scat), (const int64_t*)(w + o_sprefix), (int)scatter.size(),
                    sprefix.back(), {w + o_c, out.data()}, src64, src64 ? 1 : 0, s);
}

}  // namespace symten
