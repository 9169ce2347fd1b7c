// Internal declarations of the MI355X FMM library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fmm.h"

namespace fmm {

constexpr int kMaxLevel = 21;       // 63-bit Morton keys, 21 bits per axis
constexpr int kMaxP = 16;
constexpr int kTileN = 64;          // M2L target cells per tile (GEMM N dimension)
constexpr int kEntriesPerWork = 48; // M2L (tile, operator) entries per work item (split-K)
constexpr int kP2PThreads = 256;    // near-field workgroup; a split leaf has at most this many targets
constexpr int64_t kP2PPieceWork = int64_t(1) << 20;   // near-field interactions per piece of a split leaf
constexpr int kP2PMaxPieces = 4096;

// Coefficient count of order p and its padded length (multiple of 16: MFMA 16x16x4 blocking).
inline int ncoef(int p) { return (p + 1) * (p + 1); }
inline int ncoef_pad(int p) { return (ncoef(p) + 15) / 16 * 16; }

// Error raised inside the library; converted to fmm_status at the ABI.
struct Error {
    fmm_status status;
    std::string msg;
};
[[noreturn]] void fail(fmm_status s, const std::string &msg);
void check_hip(hipError_t e, const char *what);
#define HIP_CHECK(x) ::fmm::check_hip((x), #x)

// Host-visible results without a staging copy.  A mailbox is pinned, coherent host
// memory mapped into the device address space: a kernel writes its small result there
// and then, after a system-scope fence, a ticket; the host spins on the ticket.  Uploads
// go through the same pinned memory (an arena reset at the start of each plan build).
struct Mailbox {
    static constexpr int64_t kPostBytes = int64_t(64) << 10;   // area kernels post to (coherent)
    static constexpr int64_t kFetchBytes = int64_t(4) << 20;   // copy destination (pinned, cached)
    static constexpr int64_t kUploadBytes = int64_t(4) << 20;  // upload arena (pinned, cached)
    volatile uint64_t *host = nullptr;   // word 0: ticket; data from byte 64
    uint64_t *dev = nullptr;             // the same memory as seen by the device
    char *fetch_host = nullptr;          // pinned read-back area
    char *upload_host = nullptr;         // pinned upload arena
    int64_t upload_used = 0;
    uint64_t ticket = 0;
    uint64_t *flag_dev() const { return dev; }
    template <class T> T *data_dev() const { return reinterpret_cast<T *>(reinterpret_cast<char *>(dev) + 64); }
    template <class T> const T *data_host() const {   // read only after wait() returned
        return reinterpret_cast<const T *>(const_cast<const char *>(reinterpret_cast<const volatile char *>(host)) + 64);
    }
    uint64_t next_ticket() { return ++ticket; }
    // Spin until the ticket arrives; fails if the stream reports an error or completes
    // without delivering it.
    void wait(uint64_t t, hipStream_t s);
    // Copy n bytes of host data into the upload arena and queue their transfer to dst.
    void upload(void *dst, const void *src, size_t n, hipStream_t s);
    // Device-to-host copy of n bytes (at most kFetchBytes) into the fetch area (pinned: no
    // staging), then a stream synchronisation; returns the host copy, valid until the next
    // fetch.
    const void *fetch(const void *src, size_t n, hipStream_t s);
};
Mailbox *mailbox_acquire();        // from a process-wide pool
void mailbox_release(Mailbox *m);
struct MailboxLease {               // scope guard
    Mailbox *m = mailbox_acquire();
    ~MailboxLease() { mailbox_release(m); }
};

// Device side of a mailbox post: the data stores of this thread are made visible at
// system scope, then the ticket is written.  Every thread that wrote data must call
// mailbox_fence() before a barrier that precedes the post.
__device__ inline void mailbox_fence() { __threadfence_system(); }
__device__ inline void mailbox_post(uint64_t *flag, uint64_t ticket) {
    __threadfence_system();
    __hip_atomic_store(flag, ticket, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Workspace allocation through the plan's allocator; everything is released at destroy.
struct Alloc {
    fmm_alloc_fn alloc = nullptr;
    fmm_free_fn release = nullptr;
    void *ctx = nullptr;
    hipStream_t stream = nullptr;
    std::vector<std::pair<void *, size_t>> live;   // blocks held, with their requested sizes
    int64_t bytes = 0;                              // sum of the sizes of the blocks held
    Mailbox *mb = nullptr;   // set while a plan is built: scan totals come back through it
    void *get(size_t bytes);
    template <class T> T *get_n(int64_t n) { return static_cast<T *>(get(sizeof(T) * (size_t)(n > 0 ? n : 1))); }
    void put(void *p);       // release one allocation early
    void release_all();
};

// ---------------------------------------------------------------- primitives
// Exclusive scan of n values; returns the total (waits for it: through the allocator's
// mailbox when it has one, else by a read-back).
int64_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, Alloc &a, hipStream_t s);
int64_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, Alloc &a, hipStream_t s);
// The same without waiting: the total is written to device memory.
void exclusive_scan_i32_to(const int32_t *in, int32_t *out, int64_t n, int64_t *tot_dev, Alloc &a, hipStream_t s);
void exclusive_scan_i64_to(const int64_t *in, int64_t *out, int64_t n, int64_t *tot_dev, Alloc &a, hipStream_t s);
// Stable LSD radix sort of (key, value) on the low `bits` key bits.  The sorted data end
// in one of two buffer pairs; keys/vals are updated to point at it and the other pair
// goes back to the allocator (no copy).
void radix_sort_u64(uint64_t *&keys, int32_t *&vals, int64_t n, int bits, Alloc &a, hipStream_t s);
// Copy `bytes` (a multiple of 4, at most kPostBytes) of device memory into the mailbox's
// post area and post the ticket.
void publish(const void *src, int64_t bytes, Mailbox &m, uint64_t ticket, hipStream_t s);
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void fill_f32(float *p, float v, int64_t n, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);
template <class T> T read_back(const T *dev, hipStream_t s) {
    T v;
    HIP_CHECK(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return v;
}

// ---------------------------------------------------------------- operators
// Device operator tables for expansion order p.  Matrices are FP32 [RP][KP] row-major
// (rows = output coefficient), stored in the scaled basis described in operators.cpp.
struct OpTables {
    int p = -1;
    const uint64_t *m2m_ptrs = nullptr;   // [8] device pointers of the octant M2M matrices [KP][KP]
    const uint64_t *l2l_ptrs = nullptr;   // [8] device pointers of the octant L2L matrices [KP][KP]
    const double *m2m64_t = nullptr;      // [8][KP in][KP out] FP64, transposed (root levels)
    const double *l2l64_t = nullptr;      // [8][KP in][KP out] FP64, transposed
    const uint64_t *m2m64_ptrs = nullptr; // [8] pointers into m2m64_t
    const uint64_t *l2l64_ptrs = nullptr; // [8] pointers into l2l64_t
    const float *nu = nullptr;            // [KP] FP16 normalisation of multipole coefficients
};
const OpTables &op_tables(int p);
// Device pointers (as uint64) of the M2L operator of every key, FP32 and split-FP16 forms.
// keys: packed (level difference, offset) keys.  Creates missing operators.
void m2l_operator_ptrs(int p, const std::vector<uint64_t> &keys, std::vector<uint64_t> &f32_ptrs,
                       std::vector<uint64_t> &f16_ptrs, bool need_f16);
// Variable-order M2L: for every key (whose operator exists), the 16x16 blocks of the
// operator that are kept at tolerance tol, as one row mask per row block (bit c: k chunk c
// is kept) followed by their union ([nkeys][KP/16 + 1]), and the kept fraction of blocks.  Blocks are dropped smallest first while
// their summed weighted size stays within tol of the interaction's monopole term.
void m2l_block_rows(int p, const std::vector<uint64_t> &keys, double tol, std::vector<uint32_t> &rows,
                    std::vector<float> &kept);
// SVD-compressed M2L: for every key, device pointers of its factors Qf ([rp][KP]) and Pf
// ([KP][rp]) at ptrs[2 i], ptrs[2 i + 1], the rank kept and its padding to a multiple of 16
// (singular values of the bound-weighted operator above tol * sigma_1 are kept).
void m2l_svd_ptrs(int p, const std::vector<uint64_t> &keys, double tol, std::vector<uint64_t> &ptrs,
                  std::vector<int32_t> &rank_pad, std::vector<int32_t> &rank);
// FP64 M2L operators ([KP in][KP out], transposed) of the given keys.
void m2l_operator_ptrs64(int p, const std::vector<uint64_t> &keys, std::vector<uint64_t> &f64_ptrs);
constexpr int kRootLevels = 4;     // mixed precision: levels 0..3 keep FP64 coefficients

// M2L key packing: dl = level(source) - level(target) in [-31, 31]; offset = (c_B - c_A)
// in units of the finer cell's half side, each component in [-2^18, 2^18).
constexpr int kKeyOffBits = 19;
constexpr int64_t kKeyOffBias = int64_t(1) << 18;
__host__ __device__ inline uint64_t pack_key(int dl, int64_t nx, int64_t ny, int64_t nz) {
    return (uint64_t(dl + 32) << 57) | (uint64_t(nx + kKeyOffBias) << 38) |
           (uint64_t(ny + kKeyOffBias) << 19) | uint64_t(nz + kKeyOffBias);
}
inline void unpack_key(uint64_t k, int &dl, int64_t &nx, int64_t &ny, int64_t &nz) {
    dl = int(k >> 57) - 32;
    nx = int64_t((k >> 38) & ((1u << 19) - 1)) - kKeyOffBias;
    ny = int64_t((k >> 19) & ((1u << 19) - 1)) - kKeyOffBias;
    nz = int64_t(k & ((1u << 19) - 1)) - kKeyOffBias;
}

// ---------------------------------------------------------------- eval launchers
struct EvalArgs;   // defined in eval.hip

}  // namespace fmm

// Grouped-GEMM tables of a translation that runs level by level (M2M, L2L).
struct LevelGemm {
    int64_t ntiles = 0;
    int32_t *tile_targets = nullptr;   // [ntiles][kTileN]
    int32_t *entry_key = nullptr;      // operator (octant) of each entry
    int32_t *entry_src = nullptr;      // [entries][kTileN]
    int4 *work = nullptr;              // [ntiles] one work item per tile
    std::vector<int32_t> bucket_tile;  // first tile of each (level, octant) bucket, size kBuckets + 1
};

// --------------------------------------------------------------------- the plan
struct fmm_plan_s {
    double m2l_tol = 0.0;        // variable-order M2L tolerance (0: dense operators)
    double svd_tol = 0.0;        // SVD-compressed M2L tolerance (0: dense operators)
    const uint64_t *key_svd = nullptr;  // [nkeys][2] device pointers of the SVD factors (Qf, Pf)
    int32_t *key_rank = nullptr;        // [nkeys] padded rank of each key's factors
    double svd_rank_mean = 0.0;         // pair-weighted mean rank kept
    int lists = 0;               // 0: dual traversal; 1: level skip (one cell split at a time)
    double m2l_kept = 1.0;       // pair-weighted fraction of operator blocks applied
    uint32_t *key_rows = nullptr; // [nkeys][KP/16 + 1] kept k-chunk masks per row block, then their union
    int device = 0;
    int64_t n = 0;
    int64_t nsrc = 0, ntgt = 0;  // separate target set: n = nsrc + ntgt points, sources first (ntgt = 0: one set)
    float *tmp_u = nullptr;      // [5n] union-sized inputs of the target-set calls (charges, weights, gradients)
    float *tmp_o = nullptr;      // [11n] union-sized outputs of the target-set calls (phi, grad, dq, dx, grad psi)
    int ncrit = 0, p = 0;
    float theta = 0;
    fmm_precision prec = FMM_PREC_FP32;
    int KP = 0;                 // padded coefficient count
    fmm::Alloc mem;
    hipStream_t side = nullptr; // second stream for the near field
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    // geometry
    int k = 0;
    double x0[3] = {0, 0, 0};

    // bodies in Morton order
    int32_t *perm = nullptr;     // sorted position -> input index
    int32_t *iperm = nullptr;    // input index -> sorted position
    float4 *bodies = nullptr;    // (x, y, z, q) ; q written by each eval
    uint64_t *keys = nullptr;    // sorted keys

    // cells, level by level (Morton order inside a level)
    int64_t ncells = 0, nleaves = 0;
    int max_level = 0;
    std::vector<int64_t> level_off;  // host copy, size max_level + 2
    int32_t *c_level = nullptr, *c_start = nullptr, *c_count = nullptr, *c_parent = nullptr;
    int32_t *c_child0 = nullptr, *c_nchild = nullptr;
    int32_t *c_ix = nullptr, *c_iy = nullptr, *c_iz = nullptr;
    uint64_t *c_prefix_dev = nullptr;
    int32_t *leaves = nullptr;       // leaf cell ids, in cell order
    int32_t *leaf_id = nullptr;      // cell -> leaf index or -1
    int32_t *body_leaf = nullptr;    // [n] sorted position -> leaf cell

    // M2L
    int64_t nm2l = 0, nkeys = 0, ntargets = 0, ntiles = 0, nentries = 0, nwork = 0;
    int2 *m2l_pairs = nullptr;       // (target, source), grouped by (tile, key, lane)
    const uint64_t *key_f32 = nullptr;   // [nkeys] device pointers of FP32 operators
    const uint64_t *key_f16 = nullptr;   // [nkeys] device pointers of split-FP16 operators
    int32_t *tile_targets = nullptr;     // [ntiles][kTileN], -1 = empty lane
    int32_t *entry_key = nullptr;        // [nentries] key id
    int32_t *entry_src = nullptr;        // [nentries][kTileN] source cell or -1
    uint8_t *entry_mask = nullptr;       // [nentries] bit b: column block b (lanes 16b..16b+15) has a source
    int4 *work = nullptr;                // [nwork] (tile, entry begin, entry end, partial slot + 1 or 0 = direct)
    int64_t npartial = 0;                // work items that write a partial tile
    int32_t *tile_work = nullptr;        // [ntiles + 1] range of each tile in tile_work_idx
    int32_t *tile_work_idx = nullptr;    // [nwork] work items of each tile
    int64_t nkeys_same = 0, nm2l_same = 0;
    // M2L slot pool: pairs of sparse (tile, key) cells, regrouped by the cell pair that produced
    // them; every slot writes a partial column, summed per target in slot order
    int64_t npool = 0, nslots = 0, nslot_tiles = 0, nruns = 0;
    int64_t *slot_pos = nullptr;         // [nslots] partial column of each slot
    int32_t *run_first = nullptr;        // [nruns + 1] first slot of each target's run
    int32_t *run_tgt = nullptr;          // [nruns] target cell of each run
    LevelGemm m2m, l2l;

    // P2P
    int64_t np2p = 0, nseg = 0, p2p_interactions = 0;
    int2 *p2p_pairs = nullptr;       // (target leaf cell, source leaf cell), sorted
    int32_t *seg_off = nullptr;      // [nleaves + 1] per target leaf (leaf order)
    int2 *segs = nullptr;            // (body start, body count) runs of source bodies, self excluded
    int64_t *run_pre = nullptr;      // [nseg + 1] exclusive prefix of the run lengths
    int4 *p2p_items = nullptr;       // (leaf, piece, pieces, first partial block or -1), leaf order
    int64_t np2p_items = 0, np2p_part = 0;   // work items; partial blocks of split leaves
    float4 *p2p_part = nullptr;      // [np2p_part][kP2PThreads] partial (potential, gradient)
    float *p2p_part_h = nullptr;     // [np2p_part][kP2PThreads][6] partial Hessian (allocated on first use)

    // eval workspace
    float *M = nullptr, *L = nullptr;          // [ncells][KP]
    // mixed precision: FP64 coefficients of the root levels (cells [0, nroot))
    int64_t nroot = 0, ntiles_root = 0, nwork64 = 0;
    double *Md = nullptr, *Ld = nullptr;        // [nroot][KP]
    const uint64_t *key_f64 = nullptr;          // [nkeys] FP64 operators (0 where unused)
    int4 *work64 = nullptr;                     // work items over the root tiles
    int32_t *tile_work64 = nullptr, *tile_work_idx64 = nullptr;
    double *partial64 = nullptr;
    _Float16 *Mh = nullptr, *Ml = nullptr;      // [ncells][KP] split FP16 multipoles (normalised)
    float *Msinv = nullptr;                     // [ncells] inverse power-of-two scale of each cell
    float *partial = nullptr;                   // [nwork][kTileN][KP]
    float4 *far4 = nullptr, *near4 = nullptr;   // sorted order: (potential, gradient) of far and near field
    float *farh = nullptr, *nearh = nullptr;    // sorted order: Hessian (xx yy zz xy xz yz), allocated on first use
    bool hess_on = false;                       // the running evaluation also produces the Hessian
    float *tmp_phi = nullptr, *tmp_grad = nullptr, *tmp_gfwd = nullptr;   // adjoint scratch (input order)
    float *tmp_h = nullptr;                     // adjoint through grad phi: Hessian of the forward field
    // dipole sources (sorted order, .xyz), the bodies with one dipole component as charge,
    // and the three leaf multipoles of those charges; allocated on first use
    float4 *dip = nullptr, *dipb = nullptr;
    float *Mdip = nullptr;
    bool dip_on = false;                        // the running evaluation has dipole sources
    std::vector<hipStream_t> streams_used;       // every stream the plan's memory was used on
    int fp64_levels = 0;                        // levels 0..fp64_levels-1 kept in FP64 (mixed)

    // timing
    bool timing = false;
    hipEvent_t ev[2 * FMM_NUM_PHASES] = {};
    bool ev_valid = false;

    fmm_stats stats{};
};
