/*
 * symten — block-sparse symmetric tensors and one CTM environment move on
 * AMD Instinct MI355X (gfx950).
 *
 * A tensor is a direct sum of dense blocks, one per tuple of charge labels
 * that obeys the abelian addition rule (Sec. 2, Eq. tensor-blocks and the
 * rank-2 example): sum over legs of dir * q == flux, dir = +1 for an
 * incoming and -1 for an outgoing leg.  A contraction pairs the blocks whose
 * labels agree on the contracted legs and multiplies their dense parts
 * (Sec. 2, contraction rule r_k = m_t . m_s); results with equal open labels
 * are summed in place (Sec. 2, grouping by output quantum numbers).
 *
 * SU(2) tensors (Sec. 2, Eq. tensor-cgc: each block is a reduced tensor
 * times a generalised Clebsch-Gordan tensor) carry one doubled spin 2j per
 * leg and one coupling tree per block: the incoming legs, in leg order, are
 * coupled left to right by Clebsch-Gordan coefficients (Condon-Shortley
 * phase) to a total spin K, the outgoing legs likewise to the same K, and
 * the block's basis tensor is c[m..] = sum_M C_in(m_in; K M) C_out(m_out; K M).
 * The tree labels are (in-chain intermediate spins, out-chain intermediate
 * spins, K), all doubled.  Contracting two such tensors multiplies the
 * reduced blocks and expands each product of basis tensors in the output's
 * basis; the expansion coefficients (recoupling scalars) are computed on the
 * host in FP64 when the contraction is planned and scale the gathered A
 * operands (Sec. 2, reduction of blocks with parallel CGCs).
 *
 * Conventions shared by every entry point:
 *  - U(1) charges are integers in units of 2*S^z; Z2 labels are parities
 *    0, 1 (every charge sum taken mod 2; flux 0 or 1); SU(2) labels are
 *    doubled spins 2j (0..64) and an SU(2) tensor's flux must be 0 (Sec. 2:
 *    no quantum-number shift inside a tensor), else SYMTEN_E_SYM.
 *  - SU(2) sector dims are multiplet counts (reduced dims); a multiplet of
 *    spin j holds 2j+1 states.  Tensor algebra, the double layer, the
 *    corner and the move take all three groups; the entry points that say
 *    otherwise below (the batched corners, expectation values, unit cells,
 *    the single-layer corner: U(1) and Z2) return SYMTEN_E_UNSUPPORTED or
 *    SYMTEN_E_INVAL for SU(2); all operands of one call must share the group
 *    (SYMTEN_E_SYM otherwise).
 *  - A leg's sectors are given as parallel arrays (label, reduced dim); the
 *    library sorts them by label ascending, which fixes the state order.
 *  - Canonical block order is lexicographic in the labels, leg 0 slowest.
 *    symten_upload / symten_download exchange values in that order,
 *    row-major inside each block.
 *  - Device storage: one buffer per tensor owned by the library.  Blocks are
 *    strided views into it (symten_block_info reports offset and strides in
 *    elements); tensors made by symten_create are contiguous row-major.
 *  - Every call that takes a `stream` enqueues its device work on that HIP
 *    stream (NULL = the default stream) and returns without waiting, unless
 *    documented otherwise.  Calls that overlap on one tensor race.
 *  - Work buffers of the library's own pool that a call releases (panels,
 *    intermediates, freed tensors) go to a later call on another stream
 *    only behind an event recorded on the releasing stream, so calls on
 *    different streams never share a buffer in flight.  A tensor made on one
 *    stream and read on another is ordered by the caller, as any
 *    stream-ordered data.
 *  - Every function returns 0 (SYMTEN_OK) or a negative status; the message
 *    of the last failure on the calling thread is symten_last_error().  No
 *    C++ exception crosses this interface.
 */
#ifndef SYMTEN_H
#define SYMTEN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SYMTEN_OK              0
#define SYMTEN_E_INVAL        -1  /* bad argument, null handle, bad shape */
#define SYMTEN_E_LEGS         -2  /* contracted legs not dual (direction or sectors) */
#define SYMTEN_E_SYM          -3  /* symmetry rule violated (e.g. SU(2) flux != 0) */
#define SYMTEN_E_NOMEM        -4  /* device or host allocation failed */
#define SYMTEN_E_HIP          -5  /* a HIP runtime call failed */
#define SYMTEN_E_LINALG       -6  /* QR/SVD failed, NaN/Inf met, nothing kept */
#define SYMTEN_E_CAPACITY     -7  /* a fixed-size limit was exceeded */
#define SYMTEN_E_UNSUPPORTED  -8  /* valid request not implemented */
#define SYMTEN_E_NODEVICE     -9  /* the call needs a GPU and none is usable */

/* ---- enums ------------------------------------------------------------ */
#define SYMTEN_U1   1
#define SYMTEN_SU2  2
#define SYMTEN_Z2   3

#define SYMTEN_IN   1
#define SYMTEN_OUT -1

/* storage element type */
#define SYMTEN_F64  0
#define SYMTEN_F32  1

/* arithmetic of the sector products:
 * F64    - FP64 MFMA (storage F64)
 * F32    - FP32 MFMA (storage F32)
 * BF16   - operands rounded to bf16, FP32 accumulation (storage F32)
 * BF16X3 - each FP32 operand split x = hi + lo (hi = bf16(x),
 *          lo = bf16(x - hi)); product hi*hi + hi*lo + lo*hi on bf16 MFMA
 *          with FP32 accumulation (storage F32); about 2^-16 relative per
 *          product, which meets 1e-5 on corners but not on a whole move
 * BF16X6 - each FP32 operand split x = hi + mid + lo (mid = bf16(x - hi),
 *          lo = bf16(x - hi - mid), an exact split of the FP32 value);
 *          product hi*hi + hi*mid + mid*hi + mid*mid + hi*lo + lo*hi on
 *          bf16 MFMA with FP32 accumulation (storage F32): FP32-level
 *          accuracy at six bf16 products                                    */
#define SYMTEN_PREC_F64     0
#define SYMTEN_PREC_F32     1
#define SYMTEN_PREC_BF16    2
#define SYMTEN_PREC_BF16X3  3
#define SYMTEN_PREC_BF16X6  4

#define SYMTEN_MAX_RANK 8

typedef struct symten_tensor* symten_t;
typedef struct ctm_env* ctm_env_t;

/* Tensor description.  `labels` and `dims` are the concatenation over legs
 * of each leg's sector list; leg l owns nsec[l] consecutive entries.
 * Sectors of dim 0 are ignored; labels within a leg must be distinct.      */
typedef struct {
    int group;          /* SYMTEN_U1, SYMTEN_SU2 or SYMTEN_Z2               */
    int rank;           /* 1 .. SYMTEN_MAX_RANK                             */
    const int* dirs;    /* [rank] SYMTEN_IN / SYMTEN_OUT                    */
    const int* nsec;    /* [rank] number of sectors per leg                 */
    const int* labels;  /* [sum nsec] U(1) charge (units of 2 S^z); Z2
                           parity 0, 1; SU(2) doubled spin 2j              */
    const int* dims;    /* [sum nsec] reduced sector dimension (>= 0)       */
    int flux;           /* U(1): sum dir*q of every block; Z2: that sum
                           mod 2 (0 or 1); SU(2): 0                         */
    int dtype;          /* SYMTEN_F64 or SYMTEN_F32                         */
} symten_desc;

/* ---- tensors (Sec. 2, Eq. tensor-blocks) ------------------------------ */

/* Enumerate the allowed blocks (canonical order) and allocate a zeroed
 * device buffer holding them contiguously.  Needs a GPU.                   */
int symten_create(symten_t* out, const symten_desc* d, void* stream);

/* Same enumeration without any device memory: the handle answers the
 * metadata queries below and can be used for planning (symten_plan_info),
 * but every device operation on it fails with SYMTEN_E_INVAL.  Runs on a
 * host without a GPU.                                                      */
int symten_create_meta(symten_t* out, const symten_desc* d);

void symten_destroy(symten_t t);

int symten_rank(symten_t t, int* rank);
int symten_flux(symten_t t, int* flux);
int symten_dtype(symten_t t, int* dtype);
/* sectors of one leg: labels/dims must hold at least *nsec entries; pass
 * NULL to query the count only.                                             */
int symten_leg_info(symten_t t, int leg, int* dir, int* nsec, int* labels, int* dims);
int symten_num_blocks(symten_t t, int64_t* n);
/* total number of stored block elements (sum of block sizes)              */
int symten_nnz(symten_t t, int64_t* n);
/* block i in canonical order: labels[rank], shape[rank], offset and
 * strides[rank] in elements of the device buffer.                           */
int symten_block_info(symten_t t, int64_t i, int* labels, int* shape,
                      int64_t* offset, int64_t* strides);
/* SU(2) coupling-tree labels of block i (in-chain intermediates, out-chain
 * intermediates, total spin K; doubled).  `tree` must hold rank entries;
 * *ntree = 0 for U(1) tensors.  Either pointer may be NULL.                */
int symten_block_tree(symten_t t, int64_t i, int* ntree, int* tree);
/* Clebsch-Gordan coefficient <j1 m1; j2 m2 | J M> (Condon-Shortley phase),
 * every argument doubled, as used by the SU(2) planner (Racah's sum in
 * extended precision).  Spins 0..64 (J 0..128); 0 outside the selection
 * rules.                                                                   */
int symten_su2_cg(int tj1, int tm1, int tj2, int tm2, int tJ, int tM, double* value);
/* Expand an SU(2) tensor into the U(1) tensor of its S^z components: leg
 * charges 2m, flux 0; inside a charge sector the states are ordered by spin
 * ascending, then multiplet index; each element is the sum over the block's
 * coupling trees of reduced value times basis-tensor entry (Sec. 2, Eq.
 * tensor-cgc).  The new handle owns a new buffer of the input's dtype.
 * Waits for `stream` before returning.                                      */
int symten_su2_to_u1(symten_t* out, symten_t in, void* stream);
/* device buffer and its size in elements (>= nnz when blocks are strided). */
int symten_device_ptr(symten_t t, void** ptr, int64_t* elems);
/* Bytes of t's device buffer (elements times the storage size).           */
int symten_nbytes(symten_t t, int64_t* bytes);

/* Device memory from a caller's allocator (e.g. a framework's caching
 * allocator): alloc(bytes, ctx) returns device memory of at least `bytes`
 * (null: SYMTEN_E_NOMEM), free(ptr, bytes, ctx) releases it with the same
 * byte count.  Buffers live until their last tensor or cached plan lets go,
 * and are used on the streams passed to the library's calls, in stream
 * order, so an allocator that tracks streams should serve those streams.
 * Pass two nulls to return to the library's own caching pool.  A buffer is
 * handed back only while the registration that made it is the current one;
 * after any later call of this function it is kept until the process ends
 * (so the caller can drop an allocator that is going away, e.g. at
 * interpreter exit, by registering nulls first).  alloc and free may be
 * called from the library's own host threads (the projector stage of a move
 * enqueues from several), so they must be thread-safe.  Errors:
 * SYMTEN_E_INVAL when only one of alloc and free is null.  Not for calls in
 * flight.                                                                   */
int symten_set_allocator(void* (*alloc)(size_t bytes, void* ctx),
                         void (*free_fn)(void* ptr, size_t bytes, void* ctx), void* ctx);

/* Host FP64 values in canonical block order, row-major inside each block,
 * `n` = nnz.  Values are rounded to the storage type (round to nearest).
 * Synchronous with respect to the host buffer.                             */
int symten_upload(symten_t t, const double* values, int64_t n, void* stream);
int symten_download(symten_t t, double* values, int64_t n, void* stream);

/* ---- block-sparse contraction (Sec. 2, contraction rule) -------------- */

typedef struct {
    int64_t pairs;        /* matched block pairs                             */
    int64_t out_blocks;   /* output blocks reached by at least one pair      */
    int64_t useful_flops; /* sum over pairs of 2*m*n*k                       */
    int64_t groups;       /* dense charge-sector GEMMs the pairs fuse into   */
    int64_t gemm_flops;   /* flops of those GEMMs incl. structural zeros     */
    int64_t max_m, max_n, max_k;
} symten_plan_stats;

/* Contract legs legsA[i] of A with legsB[i] of B (i < ncon).  The output
 * legs are A's open legs then B's open legs (each in their order), then
 * permuted: output leg j is that list's entry out_perm[j] (NULL = identity).
 * Contracted legs must have opposite directions and identical sector lists,
 * else SYMTEN_E_LEGS.  Zero matched pairs is valid (a tensor without
 * blocks).  `prec` must suit both storage types (F64 needs F64 storage,
 * the others F32).  Output flux = flux(A) + flux(B).                       */
int symten_contract(symten_t* out, symten_t A, symten_t B, int ncon,
                    const int* legsA, const int* legsB, const int* out_perm,
                    int prec, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * contraction of symten_contract written into the caller's tensor `out`,
 * which holds the output's legs (A's open legs then B's, permuted by
 * out_perm), flux A.flux + B.flux and storage type, with contiguous blocks
 * (as symten_create makes them; blocks that no pair reaches are set to 0).
 * The gathered operand panels, the charge-sector products and the kernels'
 * descriptors use a fixed work area of SYMTEN_NOALLOC_SCRATCH_BYTES that
 * each GPU the library runs on holds until the process ends; no device
 * memory is allocated (the call's host-side planning uses host memory).
 * The work area's device address is looked up on the first call on each
 * device.  Every call on one GPU shares the work area and finds it as the
 * last call left it: calls that overlap on one GPU race, so issue them on
 * one stream.  The GEMM tiles are chosen without the autotuner.  Errors:
 * SYMTEN_E_CAPACITY when the contraction needs more work area,
 * SYMTEN_E_INVAL when out's legs, flux, storage type or layout differ, and
 * the errors of symten_contract.                                           */
#define SYMTEN_NOALLOC_SCRATCH_BYTES (64u << 20)
int symten_contract_noalloc(symten_t out, symten_t A, symten_t B, int ncon, const int* legsA,
                            const int* legsB, const int* out_perm, int prec, void* stream);

/* Sector matching on the device (Sec. 2, the contraction rule and the
 * grouping by output labels), from the leg tables of A and B alone: one
 * workgroup enumerates the allowed blocks of both tensors (canonical order),
 * the matched pairs (A block i, B block j) whose labels agree on the
 * contracted legs, in lexicographic (i, j) order, and the output blocks
 * reached by at least one pair: label tuples of A's open legs then B's open
 * legs (no permutation), lexicographic.  Results go to device memory and
 * the call does not wait: pairs[p] for p < min(count, pair_cap);
 * out_labels[o * rank_out + l] for o < min(count, out_cap); counts[5] =
 * {A blocks, B blocks, pairs, output blocks, status} with status 1 when a
 * list was cut at its capacity (the counts are the full ones, so a caller
 * can size the buffers and call again).  U(1) and Z2 (SYMTEN_E_UNSUPPORTED
 * otherwise); at most 64 sectors per leg (SYMTEN_E_CAPACITY); contracted
 * legs must be dual (SYMTEN_E_LEGS).  Tensors may be metadata-only; the
 * call needs a GPU.                                                        */
typedef struct {
    int32_t a_block;    /* index of the A block in A's canonical order      */
    int32_t b_block;    /* index of the B block in B's canonical order      */
    int32_t out_block;  /* index of the output block in the output list     */
    int32_t pad_;
    int64_t flops;      /* 2 m n k of the pair                              */
} symten_pair;
int symten_match_blocks(symten_t A, symten_t B, int ncon, const int* legsA, const int* legsB,
                        symten_pair* pairs, int64_t pair_cap, int* out_labels, int64_t out_cap,
                        int64_t* counts, void* stream);

/* Host-only planning of the same contraction: fills `info` and, if `out`
 * is not NULL, a metadata-only output tensor.  No GPU needed.              */
int symten_plan_info(symten_t A, symten_t B, int ncon, const int* legsA,
                     const int* legsB, const int* out_perm,
                     symten_plan_stats* info, symten_t* out);

/* ---- double layer (Sec. 3.2: rank-4 double-layer tensor) -------------- */

/* a[L,U,R,D] = sum_s A[s,l,u,r,d] A[s,l',u',r',d'] (A real) for a rank-5 A
 * with legs (physical in, l in, u in, r out, d out).
 * U(1): each (ket, bra) pair of virtual legs becomes one leg of charge
 * q_ket - q_bra whose states are ordered by that charge, then q_ket, then
 * (i_ket, i_bra) row-major.
 * SU(2): each (ket, bra) pair becomes one multiplet leg: for every spin pair
 * (j_ket, j_bra) in lexicographic order and every J in j_ket x j_bra,
 * n_ket * n_bra multiplets of spin J, row-major in (ket, bra) multiplet; the
 * fusion map is the unitary whose blocks are sqrt((2J+1)/(2j_ket+1)) times
 * the Clebsch-Gordan basis tensor of the legs (ket dual, bra dual, fused),
 * the bra legs running opposite to the ket legs.  Synchronises `stream`.
 * Output dtype = A's dtype, flux 0.                                         */
int symten_double_layer(symten_t* a_out, symten_t A, void* stream);

/* Double layer with a one-site operator between the layers (Sec. 3's
 * expectation values): b = sum over (s_bra, s_ket) of op[s_bra * d + s_ket]
 * A[s_ket, ...] (ket) A[s_bra, ...] (bra), the legs fused as in
 * symten_double_layer; for real A, Z(b) / Z(a) = <psi|O|psi> / <psi|psi>.
 * op is host memory, d x d row-major, d = the physical dimension of A
 * (at most 8), over A's physical states in charge order.  Every non-zero
 * entry must move the charge by one amount f = q(s_bra) - q(s_ket)
 * (SYMTEN_E_SYM otherwise); b's flux is dir(phys) * f.  U(1) only.        */
int symten_double_layer_op(symten_t* b_out, symten_t A, const double* op, void* stream);

/* ---- enlarged corners -------------------------------------------------- */

/* which = 1..4.  Inputs follow the clockwise environment convention:
 * C[in, out]; T[chi_in, D2, chi_out] with D2 outgoing for T1, T4 and
 * incoming for T2, T3; a[L in, U in, R out, D out].
 *   1: ((C1 T1) T4) a -> [x1, x4, r, d]    Ta = T1, Tb = T4
 *   2: ((C2 T1) T2) a -> [x1, x2, l, d]    Ta = T1, Tb = T2
 *   3: ((C3 T3) T2) a -> [x3, x2, l, u]    Ta = T3, Tb = T2
 *   4: ((C4 T3) T4) a -> [x3, x4, u, r]    Ta = T3, Tb = T4
 * `info` (may be NULL) receives the summed plan statistics of the 3 steps. */
int symten_enlarged_corner(symten_t* out, int which, symten_t C, symten_t Ta,
                           symten_t Tb, symten_t a, int prec,
                           symten_plan_stats* info, void* stream);

/* The same corner with the site tensor absorbed as two layers (the
 * single-layer alternative of Sec. 3.2, asymptotically cheaper than the
 * double layer): A[phys, l, u, r, d] replaces a; the two D^2 legs of the
 * second step that meet a are split into (ket, bra) legs by a gather, A
 * takes the ket legs, A* (A with every leg direction reversed; A is real)
 * the bra legs and the physical leg, and the free (ket, bra) pairs are
 * fused back (a gather) into a's legs.  Same legs, order and values as
 * symten_enlarged_corner with a = symten_double_layer(A); info counts the
 * contractions' flops.  U(1) and Z2.  Synchronises `stream` at the gathers. */
int symten_enlarged_corner_single_layer(symten_t* out, int which, symten_t C, symten_t Ta,
                                        symten_t Tb, symten_t A, int prec,
                                        symten_plan_stats* info, void* stream);

/* Batched corners: n independent corner-1 contractions ((C T1) T4) a, each
 * step of all n fused into one grouped-GEMM launch.  use_graph != 0 records
 * the whole batch into a HIP graph on first use and replays it afterwards
 * (a change of input buffers drains the device and records it again).
 * out[i] receive the corners, views of one new buffer per call: results of
 * earlier calls stay valid.  The plans, panels, intermediate results and
 * the graph are cached per (n, prec, leg structures) and shared by the
 * calls with that key, so such calls must not overlap on different streams.
 * info (may be NULL) receives the summed statistics.  U(1) and Z2.          */
int symten_enlarged_corners_batched(int n, symten_t* out, const symten_t* C,
                                    const symten_t* Ta, const symten_t* Tb,
                                    const symten_t* a, int prec, int use_graph,
                                    symten_plan_stats* info, void* stream);

/* ---- CTM environment and one move ------------------------------------- */

#define CTM_LEFT   0
#define CTM_TOP    1
#define CTM_RIGHT  2
#define CTM_BOTTOM 3
#define CTM_MAX_SECTORS 64

typedef struct {
    int nsec;                        /* sectors of the new chi leg         */
    int charge[CTM_MAX_SECTORS];     /* U(1) charge, or SU(2) spin 2J      */
    int kept[CTM_MAX_SECTORS];       /* kept values (SU(2): multiplets)    */
    int n_sv_sectors;                /* sectors that had singular values   */
    int sv_charge[CTM_MAX_SECTORS];
    int sv_count[CTM_MAX_SECTORS];
    double trunc_err;                /* sum discarded s^2 / sum s^2, each
                                        SU(2) value counted 2J+1 times     */
    double gap;                      /* (s_last_kept - s_first_dropped)/s_max */
    double s_max;
    double cutoff;                   /* relative truncation floor: values
                                        <= cutoff * s_max were dropped      */
    int64_t flops_corners, flops_halves, flops_renorm; /* useful flops     */
    int64_t flops_proj;              /* FP64 flops of Y = H_u^T H_d        */
    double ms_corners, ms_halves, ms_proj, ms_renorm, ms_total;
} ctm_move_stats;

/* The environment takes its own references to C1..C4, T1..T4 (it keeps the
 * handles; do not destroy them while the environment lives).               */
int ctm_env_create(ctm_env_t* env, const symten_t C[4], const symten_t T[4]);
void ctm_env_destroy(ctm_env_t env);
/* Current tensor k: 0..3 = C1..C4, 4..7 = T1..T4.  Returns a new handle
 * (sharing the storage) that the caller releases with symten_destroy.      */
int ctm_env_get(ctm_env_t env, int k, symten_t* t);

/* One CTM move (Sec. 3, the projector scheme it cites) toward direction
 * `dir`: CTM_LEFT absorbs a column into C1, T4, C4; CTM_TOP, CTM_RIGHT and
 * CTM_BOTTOM are the left move of the network turned 1, 2 or 3 quarter turns
 * counterclockwise (C1' = C2, ..., T4' = T1, a'[l,u,r,d] = a[u,r,d,l], the
 * legs that land against the (in, in, out, out) convention reversed: a U(1)
 * relabelling, no data moves) and update C1, T1, C2 / C2, T2, C3 / C3, T3, C4.
 * SU(2): the reversed legs of the turned network go through the S^z
 * components (a reversed leg maps (j, m) to (j, -m) with the phase
 * (-1)^(j-m), then the result is projected back onto reduced blocks); the
 * half-integer spins of the T's D^2 legs, which four turns multiply by -1,
 * are set back, so the environment stays that of the caller's a.
 * The left move:
 * four enlarged corners, halves H_u = C~1 C~2 and H_d = C~4 C~3, per fused
 * sector of the left cut the singular triplets of M = R_u R_d^T (QR
 * H_u^T = Q_u R_u, H_d^T = Q_d R_d; taken from Y = H_u^T H_d, which has the
 * same singular values, with V_Y = Q_d V and U_Y = Q_u U), global truncation
 * to chi states (ties: sector, then index ascending; s <= c s_max dropped,
 * c = 1e-14 for PREC_F64; the other precisions take s from the Gram matrix
 * Y Y^T and drop s <= sqrt(N eps) s_max, eps = 2^-52 and N the order of the
 * largest block, below which that route does not resolve s; a degenerate
 * set is never split: values within a relative 1e-8 (F64), 1e-5 (F32,
 * BF16X6) or 1e-4 (BF16X3, BF16) of the last kept one are dropped with it),
 * projectors P = R_d^T V S^-1/2 = H_d V_Y S^-1/2 and
 * P~ = S^-1/2 U^T R_u = S^-1/2 U_Y^T H_u^T (largest-magnitude entry of every
 * P~ row made positive), then C1' = (C1 T1) P, T4' = P~ (T4 a) P,
 * C4' = P~ (C4 T3), each scaled to unit Frobenius norm in FP64.  `chi`
 * counts states.  U(1): sectors are fused charges.  SU(2): the two legs of
 * each side of the cut are fused by a unitary isometry into one multiplet
 * leg, sectors are its total spins J, each kept value is a multiplet of
 * 2J+1 states and multiplets are kept whole (descending, stopping at the
 * first that does not fit).  Synchronises `stream` once during the move
 * (truncation needs the singular values on the host) and returns with
 * `stream` synchronised: the updated tensors are complete on return.  The
 * eigensolves of the projector stage run on `stream` (the library's solver,
 * orders up to symten_eigh_max_order); larger ones (rocSOLVER) run on three
 * side streams of the environment, each enqueued by a short-lived host
 * thread, all joined to `stream` before the call returns.  Calls on one
 * environment must not overlap.                                             */
int ctm_move(ctm_env_t env, symten_t a, int dir, int chi, int prec,
             ctm_move_stats* st, void* stream);

/* Partition function per site of a classical model (U(1), Z2 or SU(2);
 * SU(2) networks are contracted on reduced blocks, the closing trace counting
 * a spin-j block 2j+1 times), FP64, from the environment of a 1x1 cell
 * (SYMTEN_E_INVAL for a unit cell: ctm_cell_site_partition), on a
 * block x block patch (block 1 or 2):
 * kappa^(block^2) = Z_bb Z_00 / (Z_b0 Z_0b), Z_nm the closed network of the
 * four corners with n columns and m rows of edge tensors and the n x m site
 * tensors a between them (Z_00 = Tr C1 C2 C3 C4); the boundary factors cancel
 * in the ratio.  block = 2 also cancels the corner weights when the
 * environment bonds alternate between two charge parities from site to site
 * (every D charge odd, e.g. arrow models), which bias block = 1; it needs a
 * positive ratio (SYMTEN_E_LINALG otherwise).  z (may be NULL) receives
 * Z_00, Z_b0, Z_0b, Z_bb.  Synchronous.                                      */
int ctm_site_partition(ctm_env_t env, symten_t a, int block, double* kappa, double* z, void* stream);

/* ---- unit cells (Lx x Ly sites, the paper's 2 x 2 geometry) ----------
 * Every site (x, y) (x to the right, y downwards, periodic) has its own
 * environment C1..C4, T1..T4 with the conventions of the 1x1 case, passed
 * as C[4 (x Ly + y) + i], T[4 (x Ly + y) + i] (the environment keeps
 * references to them), and its own site tensor a[x Ly + y].  U(1) and Z2.  */
int ctm_cell_create(ctm_env_t* env, int Lx, int Ly, const symten_t* C, const symten_t* T);
/* Current tensor k (0..3 = C1..C4, 4..7 = T1..T4) of site (x, y); a new
 * handle sharing the storage.                                               */
int ctm_cell_get(ctm_env_t env, int x, int y, int k, symten_t* t);
/* One move of the cell toward `dir` (Sec. 3, the scheme it cites, with one
 * projector pair per cut).  The left move runs column by column
 * (x = 0 .. Lx-1): for every cut y (between site rows y and y+1) the
 * projectors of the 1x1 move are computed from the enlarged corners of the
 * 2 x 2 block of sites (x, y), (x+1, y), (x+1, y+1), (x, y+1), each from its
 * own site's environment; then the left column of the sites (x+1, y) is
 * renormalised: C1' = P(y-1)^T C1 T1 (x, y), T4' = P~(y-1) T4 a (x, y) P(y),
 * C4' = C4 T3 (x, y) P~(y)^T, each to unit norm.  Column x+1 changes before
 * the next column is processed.  Other directions turn the cell (site
 * (x, y) -> (y, Lx-1-x), every site as in ctm_move) and back.
 * ctm_move_singular_values returns the kept values of every cut of the
 * move, cut after cut, each cut's descending.  Returns with `stream`
 * synchronised, as ctm_move does.                                          */
int ctm_cell_move(ctm_env_t env, const symten_t* a, int dir, int chi, int prec, void* stream);
/* ctm_site_partition on the environment of site (x, y).                   */
int ctm_cell_site_partition(ctm_env_t env, int x, int y, symten_t a, int block, double* kappa, double* z,
                            void* stream);

/* Expectation value on an n x m patch (n columns, m rows; 1 <= n, m <= 2)
 * of the 1x1-cell environment, FP64: value = Z_nm(sites) / Z_nm(a), where
 * Z_nm(sites) is the closed network of ctm_site_partition with the site
 * tensors replaced by sites[n*m] (row-major: row 0 on top, column 0 on the
 * left; each a rank-4 tensor of a's group (U(1) or Z2) with a's legs, any
 * flux; a patch whose fluxes do not add up to 0 gives 0).  For a PEPS, sites are double layers
 * with one-site operators between the layers (symten_double_layer_op) and
 * the value is <O_1 O_2 ...> of Sec. 3's energy evaluation; for a classical
 * model they are impurity weights.  Synchronous.                            */
int ctm_expectation(ctm_env_t env, symten_t a, int n, int m, const symten_t* sites, double* value,
                    void* stream);

/* Nearest-neighbour Heisenberg energy per bond, S_i . S_j = Sz Sz +
 * (S+ S- + S- S+)/2 (J = 1), FP64, of the state A[phys, l, u, r, d]
 * (U(1): physical charges 2m for m = -S..S, one state each; SU(2): one
 * physical multiplet of spin S; S <= 7/2; Z2: spin 1/2 with the physical
 * leg {0: 1, 1: 1} in the spin-flip parity basis (|up> +- |down>)/sqrt2,
 * where Sx keeps the parity and Sy, Sz flip it) in the current 1x1 environment,
 * which must be the environment of A's double layer: *e_h on a horizontal
 * bond (2 x 1 patch), *e_v on a vertical one.  The double layers with Sz,
 * S+, S- between the layers are built on the device
 * (symten_double_layer_op); for SU(2), whose spin operators are not
 * invariant, the state is measured through its S^z components: the
 * environment is expanded and the double layers are built in the S^z basis
 * of its fused multiplets; for Z2 the three components are summed as
 * Sx Sx + Sz Sz - J J with the real J = -i Sy.  Synchronous.               */
int ctm_heisenberg_bond_energy(ctm_env_t env, symten_t A, double* e_h, double* e_v, void* stream);

/* CTM iteration with the error estimate of Sec. 3 (U(1), Z2 or SU(2); 1x1
 * environments).  A step is one
 * move toward each of the four sides (left, top, right, bottom).  At fixed
 * chi, steps run until kappa changes by less than tol from one step to the
 * next, or max_steps steps (the value before the first step is measured
 * too); err_steps is the larger of the last two changes.  Then chi doubles,
 * continuing from the current environment, while 2 chi <= chi_max, until the
 * values at the last two chis differ by less than tol; err_chi is that
 * difference (0 with one chi).  error = max(err_steps, err_chi); kappa is the
 * value at the last chi.  The paper's settings: tol = 1e-8, max_steps = 15,
 * chi_max = 128.                                                            */
typedef struct {
    int chi;          /* first environment dimension (states) */
    int chi_max;      /* doubling stops before chi would exceed it */
    int prec;         /* SYMTEN_PREC_* of the moves */
    int block;        /* kappa estimator patch, 1 or 2 (ctm_site_partition) */
    int max_steps;    /* steps per chi */
    double tol;       /* absolute change of kappa */
} ctm_run_opts;
typedef struct {
    double kappa, err_steps, err_chi, error;
    int steps;        /* steps at the last chi */
    int total_steps;  /* steps over all chis */
    int chi;          /* last chi */
    int levels;       /* number of chis */
} ctm_run_result;
int ctm_run(ctm_env_t env, symten_t a, const ctm_run_opts* opts, ctm_run_result* result, void* stream);

/* Singular values of the last move, per sector in charge order, each
 * sector descending.  cap = capacity of `s`; *n receives the count.        */
int ctm_move_singular_values(ctm_env_t env, double* s, int64_t cap, int64_t* n);
/* Projectors of the last move as tensors (new handles, released with
 * symten_destroy): P[chi out, D2 in, k in] and P~[k out, chi in, D2 out];
 * FP64 for U(1), the move's storage type for SU(2).                         */
int ctm_move_projectors(ctm_env_t env, symten_t* P, symten_t* Pt);

/* Replace tensor k (0..3 = C1..C4, 4..7 = T1..T4) of the environment; the
 * environment keeps its own reference to t's storage.                      */
int ctm_env_set(ctm_env_t env, int k, symten_t t);

/* ---- FP64 symmetric eigensolver of the projector stage ----------------- */

/* Sec. 3 (the projector scheme it cites): every sector of a cut needs the
 * singular triplets of one matrix; ctm_move takes them from a symmetric
 * eigenproblem (the Gram matrix Y Y^T, or the Jordan-Wielandt matrix
 * [[0, Y], [Y^T, 0]] in FP64 moves), solved by these kernels: Householder
 * tridiagonalisation with the rows of each matrix held in the LDS of its own
 * workgroups (one exchange between them per column), every eigenvalue by
 * multisection of Sturm counts, eigenvectors by inverse iteration (close
 * eigenvalues reorthogonalised), back-transformation through the reflectors.
 * count problems; A[i]: device, n[i] x n[i], column-major with leading
 * dimension lda[i] >= n[i], symmetric with both triangles stored, read only
 * (row i is read as column i); w[i]: device,
 * n[i] doubles, receives every eigenvalue in ascending order; Z[i]: device,
 * n[i] x k[i] column-major (ld n[i]), receives the eigenvectors of the k[i]
 * largest eigenvalues, column j for the (j+1)-th largest, unit norm, sign
 * unspecified (k[i] = 0: values only, Z[i] may be NULL).  Buffers stay the
 * caller's.  Orders above symten_eigh_max_order fail with
 * SYMTEN_E_CAPACITY, a bad argument with SYMTEN_E_INVAL.  Synchronises
 * `stream` once, between the values and the vectors.                       */
int symten_eigh(int count, const int* n, const double* const* A, const int* lda, double* const* w,
                const int* k, double* const* Z, void* stream);
/* Largest order symten_eigh (and the projector stage's own solver) takes on
 * the current device; larger blocks of a cut go to the vendor eigensolver. */
int symten_eigh_max_order(int* nmax);

/* ---- kernel timing ------------------------------------------------------ */

/* While enabled, every gather and grouped-GEMM launch is bracketed by HIP
 * events on its stream.  symten_profile_end waits for those events and
 * returns one entry per kernel (name = kernel symbol and tile shape).       */
typedef struct {
    char name[64];
    int64_t launches;
    double ms;               /* summed event time of the launches           */
    int64_t useful_flops;    /* summed block-pair flops (GEMM kernels)      */
    int64_t gemm_flops;      /* summed flops issued incl. structural zeros   */
    int64_t bytes;           /* summed algorithmic bytes: operands read once
                                and results written once                    */
} symten_kernel_stat;

int symten_profile_begin(void);
int symten_profile_end(symten_kernel_stat* out, int cap, int* n);

/* ---- misc --------------------------------------------------------------- */
const char* symten_last_error(void);
int symten_version(void);
/* Wait for all work on `stream`.                                            */
int symten_sync(void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SYMTEN_H */
