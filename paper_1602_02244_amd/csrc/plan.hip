// Plan construction on the device: root cube and Morton keys, radix sort, adaptive
// octree (level by level), dual tree traversal with the MAC, and the grouping of the
// interaction lists into the layouts the evaluation kernels consume.
//
// Paper: hierarchical decomposition and multipole/local expansions (Sec. 1), 1-D
// Morton ordering for locality (Sec. 3.1), interaction lists from a dual tree
// traversal with a multipole acceptance criterion (Sec. 2.2), translation operators
// shared by boxes with the same relative position (Sec. 2.2).
#include <algorithm>
#include <unordered_map>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "fmm_internal.h"

namespace fmm {

// ----------------------------------------------------------------- bounding box
__global__ void __launch_bounds__(256) k_bbox_partial(const float *pts, int64_t n, float *part) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float bad = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float v = pts[3 * i + a];
            if (!isfinite(v)) bad = 1.f;
            lo[a] = fminf(lo[a], v);
            hi[a] = fmaxf(hi[a], v);
        }
    }
    __shared__ float sh[7][256];
    for (int a = 0; a < 3; ++a) { sh[a][threadIdx.x] = lo[a]; sh[3 + a][threadIdx.x] = hi[a]; }
    sh[6][threadIdx.x] = bad;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int a = 0; a < 3; ++a) {
                sh[a][threadIdx.x] = fminf(sh[a][threadIdx.x], sh[a][threadIdx.x + off]);
                sh[3 + a][threadIdx.x] = fmaxf(sh[3 + a][threadIdx.x], sh[3 + a][threadIdx.x + off]);
            }
            sh[6][threadIdx.x] = fmaxf(sh[6][threadIdx.x], sh[6][threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) part[blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_bbox_final(const float *part, int nb, float *out, uint64_t *flag,
                                                    uint64_t ticket) {
    __shared__ float sh[7][256];
    float r[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.f};
    for (int b = threadIdx.x; b < nb; b += 256) {
        for (int a = 0; a < 3; ++a) {
            r[a] = fminf(r[a], part[b * 8 + a]);
            r[3 + a] = fmaxf(r[3 + a], part[b * 8 + 3 + a]);
        }
        r[6] = fmaxf(r[6], part[b * 8 + 6]);
    }
    for (int a = 0; a < 7; ++a) sh[a][threadIdx.x] = r[a];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int a = 0; a < 3; ++a) {
                sh[a][threadIdx.x] = fminf(sh[a][threadIdx.x], sh[a][threadIdx.x + off]);
                sh[3 + a][threadIdx.x] = fmaxf(sh[3 + a][threadIdx.x], sh[3 + a][threadIdx.x + off]);
            }
            sh[6][threadIdx.x] = fmaxf(sh[6][threadIdx.x], sh[6][threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) {
        out[threadIdx.x] = sh[threadIdx.x][0];
        mailbox_fence();
    }
    __syncthreads();
    if (threadIdx.x == 0) mailbox_post(flag, ticket);
}

// Root cube: side 2^k, the smallest power of two with hi_a - x0_a <= 2^k on every axis
// (the closed box), x0_a = lo_a rounded down to a multiple of 2^(k-22); a point on the
// upper face is clamped into the last cell.  Every cell centre and centre difference is
// then an exact dyadic number (exact integer MAC, exact operator keys).
static void root_cube(const float lo[3], const float hi[3], int &k, double x0[3]) {
    double E = 0;
    for (int a = 0; a < 3; ++a) E = std::max(E, (double)hi[a] - (double)lo[a]);
    int e = 0;
    std::frexp(E, &e);
    k = e - 1;
    for (;;) {
        double unit = std::ldexp(1.0, k - 22);
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            x0[a] = std::floor((double)lo[a] / unit) * unit;
            if (!((double)hi[a] - x0[a] <= std::ldexp(1.0, k))) ok = false;
        }
        if (ok) break;
        ++k;
    }
}

// ----------------------------------------------------------------- Morton keys
__device__ inline uint64_t spread3(uint64_t v) {   // bit b -> bit 3b, 21 bits
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline uint64_t axis_coord(float x, double x0, double scale) {
    double v = floor(((double)x - x0) * scale);
    v = fmax(v, 0.0);
    v = fmin(v, (double)((1 << kMaxLevel) - 1));
    return (uint64_t)v;
}

__global__ void k_keys(const float *pts, int64_t n, double x0x, double x0y, double x0z, double scale,
                       uint64_t *keys, int32_t *vals) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t ix = axis_coord(pts[3 * i], x0x, scale);
        uint64_t iy = axis_coord(pts[3 * i + 1], x0y, scale);
        uint64_t iz = axis_coord(pts[3 * i + 2], x0z, scale);
        keys[i] = (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz);
        vals[i] = (int32_t)i;
    }
}

__global__ void k_invert_perm(const int32_t *perm, int64_t n, int32_t *iperm) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        iperm[perm[i]] = (int32_t)i;
}

__global__ void k_gather_bodies(const float *pts, const int32_t *perm, int64_t n, float4 *bodies) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = perm[i];
        bodies[i] = make_float4(pts[3 * j], pts[3 * j + 1], pts[3 * j + 2], 0.f);
    }
}

// ----------------------------------------------------------------- octree
// Leaf rule: a cell splits iff it holds more than ncrit bodies and lies above level 21.
// Children are the non-empty octants.  Eight lanes per cell: lane o finds the first body
// of octant o by binary search in the sorted keys (the seven searches run side by side
// instead of one after another), and the group exchanges its bounds by shuffles.
__global__ void k_split(int64_t ncl, const int32_t *start, const int32_t *count, const uint64_t *prefix, int level,
                        int ncrit, const uint64_t *keys, int32_t *nchild, int32_t *cstart8, int32_t *ccount8) {
    // the stride is a multiple of 8, so the eight lanes of a group stay together
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; (t >> 3) < ncl; t += stride) {
        const int64_t i = t >> 3;
        const int o = (int)(t & 7);
        const int s = start[i], c = count[i];
        const bool split = c > ncrit && level < kMaxLevel;
        int b = s;                       // first body of octant o
        if (split && o > 0) {
            const int shift = 3 * (kMaxLevel - (level + 1));
            const uint64_t want = prefix[i] * 8 + (uint64_t)o;
            int lo = s, hi = s + c;      // first position with (key >> shift) >= want
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((keys[mid] >> shift) < want) lo = mid + 1;
                else hi = mid;
            }
            b = lo;
        }
        int bn = __shfl_down(b, 1, 8);
        if (o == 7) bn = s + c;
        int nz = (split && bn > b) ? 1 : 0;
        nz += __shfl_xor(nz, 1, 8);
        nz += __shfl_xor(nz, 2, 8);
        nz += __shfl_xor(nz, 4, 8);
        if (split) {
            cstart8[i * 8 + o] = b;
            ccount8[i * 8 + o] = bn - b;
        }
        if (o == 0) nchild[i] = split ? nz : 0;
    }
}

__global__ void k_write_children(int64_t ncl, int64_t glob_base, int64_t next_base, const int32_t *nchild,
                                 const int32_t *off, const int32_t *cstart8, const int32_t *ccount8,
                                 const uint64_t *prefix, const int32_t *ix, const int32_t *iy, const int32_t *iz,
                                 int32_t *child0, uint64_t *n_prefix, int32_t *n_ix, int32_t *n_iy, int32_t *n_iz,
                                 int32_t *n_start, int32_t *n_count, int32_t *n_parent, int32_t *n_level,
                                 int32_t child_level) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= ncl) return;
    int nch = nchild[i];
    child0[i] = nch > 0 ? (int32_t)(next_base + off[i]) : -1;
    if (nch == 0) return;
    int w = off[i];
    for (int o = 0; o < 8; ++o) {
        int cc = ccount8[i * 8 + o];
        if (cc == 0) continue;
        n_prefix[w] = prefix[i] * 8 + (uint64_t)o;
        n_ix[w] = 2 * ix[i] + ((o >> 2) & 1);
        n_iy[w] = 2 * iy[i] + ((o >> 1) & 1);
        n_iz[w] = 2 * iz[i] + (o & 1);
        n_start[w] = cstart8[i * 8 + o];
        n_count[w] = cc;
        n_parent[w] = (int32_t)(glob_base + i);
        n_level[w] = child_level;
        ++w;
    }
}

__global__ void k_init_root(int32_t n, uint64_t *prefix, int32_t *ix, int32_t *iy, int32_t *iz, int32_t *start,
                            int32_t *count, int32_t *parent, int32_t *level) {
    if (threadIdx.x == 0) {
        prefix[0] = 0;
        ix[0] = iy[0] = iz[0] = 0;
        start[0] = 0;
        count[0] = n;
        parent[0] = -1;
        level[0] = 0;
    }
}

// ----------------------------------------------------------------- dual traversal
struct CellView {
    const int32_t *level, *ix, *iy, *iz, *child0, *nchild;
    const uint64_t *prefix;   // Morton prefix (key >> 3 (21 - level))
    int lists;                // 0: rule 3 splits both cells; 1: only the smaller prefix (level skip)
    // separate target set only (else null): bit 0 the cell holds a source, bit 1 a target
    const uint8_t *kind = nullptr;
};

// With a separate target set a pair of cells (A, B) carries something only when A holds a
// target and B a source (the field at the targets) or A a source and B a target (the
// adjoint, whose weights sit on the targets); a child holds a subset of its cell's bodies,
// so a pair that carries nothing has no descendant pair that does.
__device__ inline bool pair_carries(int ka, int kb) { return ((ka & 2) && (kb & 1)) || ((ka & 1) && (kb & 2)); }

// Kind of every cell of a target-set plan: counts of sources among its bodies from the
// exclusive prefix `srcpre` of the sorted bodies' source flags (srcpre[n] = total).
__global__ void k_src_flags(const int32_t *perm, int64_t n, int64_t nsrc, int32_t *flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = perm[i] < nsrc ? 1 : 0;
}
__global__ void k_cell_kind(const int32_t *start, const int32_t *count, int64_t nc, const int32_t *srcpre,
                            uint8_t *kind) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        const int s0 = start[c], k = count[c];
        const int ns = srcpre[s0 + k] - srcpre[s0];
        kind[c] = (uint8_t)((ns > 0 ? 1 : 0) | (k - ns > 0 ? 2 : 0));
    }
}

// Exclusive scan of four wave-uniform counters over the four waves of a 256-thread
// block: `off` = the counts of the waves before this one, `tot` = the block's totals.
__device__ inline void block_scan_waves4(const int (&v)[4], int (&off)[4], int (&tot)[4]) {
    __shared__ int ws[4][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < 4; ++c) ws[c][wave] = v[c];
    __syncthreads();
    for (int c = 0; c < 4; ++c) {
        off[c] = tot[c] = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wave) off[c] += ws[c][w];
            tot[c] += ws[c][w];
        }
    }
    __syncthreads();
}

__device__ inline uint64_t key_hash(uint64_t k) {   // splitmix64 finaliser
    k ^= k >> 30; k *= 0xbf58476d1ce4e5b9ull;
    k ^= k >> 27; k *= 0x94d049bb133111ebull;
    k ^= k >> 31;
    return k;
}
constexpr uint64_t kEmpty = ~0ull;

__device__ inline uint64_t pair_key(const CellView &C, int a, int b, int32_t *overflow) {
    int la = C.level[a], lb = C.level[b];
    int lf = la > lb ? la : lb;
    int64_t sa = int64_t(1) << (lf - la), sb = int64_t(1) << (lf - lb);
    // D = c_B - c_A in units of the finer half side
    int64_t nx = (2 * (int64_t)C.ix[b] + 1) * sb - (2 * (int64_t)C.ix[a] + 1) * sa;
    int64_t ny = (2 * (int64_t)C.iy[b] + 1) * sb - (2 * (int64_t)C.iy[a] + 1) * sa;
    int64_t nz = (2 * (int64_t)C.iz[b] + 1) * sb - (2 * (int64_t)C.iz[a] + 1) * sa;
    if (nx < -kKeyOffBias || nx >= kKeyOffBias || ny < -kKeyOffBias || ny >= kKeyOffBias || nz < -kKeyOffBias ||
        nz >= kKeyOffBias) {
        *overflow = 1;
        return 0;
    }
    return pack_key(lb - la, nx, ny, nz);
}

// Insert a key into the open-addressing table (linear probing, at most `mask + 1`
// probes; a full table raises flags[1]); returns its slot.
__device__ inline int32_t key_slot(uint64_t key, uint64_t *table, uint64_t mask, int32_t *flags) {
    uint64_t h = key_hash(key) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        const uint64_t cur = table[h];
        if (cur == key) return (int32_t)h;
        if (cur == kEmpty) {
            const uint64_t prev = atomicCAS((unsigned long long *)&table[h], (unsigned long long)kEmpty,
                                            (unsigned long long)key);
            if (prev == kEmpty || prev == key) return (int32_t)h;
        }
        h = (h + 1) & mask;
    }
    flags[1] = 1;
    return (int32_t)h;
}

// One traversal step.  Every pair of `front` needs a split; its child pairs (rules 3-4)
// are classified here: M2L and P2P pairs go to their lists, pairs that need a further
// split to `next`.  Each lane classifies one child pair, one block scan and one atomic
// per list reserve the ranges, then the lane writes.  Writes past a list's capacity are
// dropped; the counters still advance, so the host sees the exact sizes and repeats
// the step with larger lists.  cnt = (M2L pairs, P2P pairs, next frontier); k_trav_post
// hands them to the host after the step and clears the frontier count.
//
// Traversal rules for the pair (A, B):
//   1. MAC accepted                    -> M2L        (action 0)
//   2. else both leaves                -> P2P        (action 1)
//   3. else both split, same level     -> all child pairs; with level skip (lists = 1) only
//      the cell with the smaller Morton prefix is split, so that the other one can serve
//      the children whole when the MAC allows (the choice depends on the unordered pair,
//      which keeps the lists symmetric)
//   4. else split the coarser cell (on a tie the non-leaf) if it is not a leaf,
//      otherwise the other one.
__device__ inline void split_ranges(const CellView &C, int a, int b, int &a0, int &na, int &b0, int &nb) {
    int nca = C.nchild[a], ncb = C.nchild[b];
    int la = C.level[a], lb = C.level[b];
    bool splitA, splitB;
    if (nca > 0 && ncb > 0 && la == lb && C.lists == 0) {
        splitA = splitB = true;
    } else if (nca > 0 && ncb > 0 && la == lb) {
        splitA = C.prefix[a] <= C.prefix[b];
        splitB = !splitA;
    } else {
        if (la < lb) splitA = nca > 0;
        else if (lb < la) splitA = ncb == 0;
        else splitA = nca > 0;
        splitB = !splitA;
    }
    if (splitA) { a0 = C.child0[a]; na = nca; } else { a0 = a; na = 1; }
    if (splitB) { b0 = C.child0[b]; nb = ncb; } else { b0 = b; nb = 1; }
}

__global__ void k_trav_post(unsigned long long *cnt, unsigned long long *post, uint64_t *flag, uint64_t ticket) {
    if (threadIdx.x == 0) {
        post[0] = cnt[0];
        post[1] = cnt[1];
        post[2] = cnt[2];
        post[3] = cnt[3];
        cnt[2] = 0;
        mailbox_post(flag, ticket);
    }
}
__global__ void k_set_counters(unsigned long long *cnt, int64_t nm, int64_t np, int64_t nr) {
    if (threadIdx.x == 0) {
        cnt[0] = (unsigned long long)nm;
        cnt[1] = (unsigned long long)np;
        cnt[2] = 0;
        cnt[3] = (unsigned long long)nr;
    }
}

// Each wave takes kTravPerWave frontier pairs in turn, one lane per child pair (at most
// 8 x 8); the frontier pair and its split are wave-uniform; the data of the children are
// loaded once (lanes 0-7: children of A, lanes 8-15: children of B) and passed on by
// cross-lane shuffles.  Outputs are written in (wave, frontier pair, lane) order, so
// that the lanes of one store write consecutive words and the M2L pairs of one target
// child (lanes 8x .. 8x+7) are consecutive: such a group is a slot, and one record per
// slot is written beside the pairs; it also marks its target.  An M2L pair enters its
// operator key into the key table (the table slot is stored beside the pair).
//
// Slot record {target, first pair, b0, info}: the slot's pairs are (target, b0 + y) for the
// set bits y of its source mask, stored from `first` on in increasing y; b0 is the first
// child of the frontier pair's source cell B when B was split, else B.  info: bits 0-1 how
// the frontier pair was split (bit 0 target side, bit 1 source side), bits 2-9 the source
// mask, bits 10-12 the target's octant, bits 13-20 the octants of B's children (child y
// has the y-th lowest of them: children are stored in Morton digit order, which is the
// octant order).
struct TravOut {
    int2 *m2l;
    int32_t *m2l_slot;
    int64_t cap_m;
    int4 *rec;            // slot records {target, first pair, b0, info}
    int64_t cap_r;
    int2 *p2p;
    int64_t cap_p;
    int2 *next;
    int64_t cap_n;
    uint64_t *table;      // operator-key table, mask + 1 slots
    uint64_t mask;
    int32_t *flags;       // key out of range, table full
    int32_t *is_target;   // [ncells] the cell is the target of an M2L pair
};
constexpr int kTravPerWave = 8;
__global__ void __launch_bounds__(256) k_trav_step(CellView C, const int2 *front, int64_t nf, double theta2,
                                                   unsigned long long *cnt, TravOut o) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t f0 = (blockIdx.x * (int64_t)(blockDim.x >> 6) + wave) * kTravPerWave;
    const int lane = threadIdx.x & 63, x = lane >> 3, y = lane & 7;
    int pa[kTravPerWave], pb[kTravPerWave], act[kTravPerWave], src0[kTravPerWave], info[kTravPerWave];
    uint64_t key[kTravPerWave];
    int cw[4] = {0, 0, 0, 0};   // this wave's M2L pairs, P2P pairs, next pairs, slot records
#pragma unroll
    for (int k = 0; k < kTravPerWave; ++k) {
        const int64_t f = f0 + k;
        pa[k] = pb[k] = 0;
        act[k] = -1;
        key[k] = 0;
        info[k] = 0;
        src0[k] = 0;
        if (f < nf) {
            int a0, na, b0, nb;
            const int2 pr = front[f];
            const int ga = __builtin_amdgcn_readfirstlane(pr.x), gb = __builtin_amdgcn_readfirstlane(pr.y);
            split_ranges(C, ga, gb, a0, na, b0, nb);
            src0[k] = b0;
            const bool ld = lane < 8 ? lane < na : (lane < 16 && lane - 8 < nb);
            const int cell = lane < 8 ? a0 + lane : b0 + (lane - 8);
            int lv = 0, cx = 0, cy = 0, cz = 0, ch = 0, kd = 3;
            if (ld) {
                lv = C.level[cell];
                cx = C.ix[cell];
                cy = C.iy[cell];
                cz = C.iz[cell];
                ch = C.nchild[cell];
                if (C.kind) kd = C.kind[cell];
            }
            const int la = __shfl(lv, x, 64), ax = __shfl(cx, x, 64), ay = __shfl(cy, x, 64), az = __shfl(cz, x, 64),
                      ca = __shfl(ch, x, 64);
            const int lb = __shfl(lv, 8 + y, 64), bx = __shfl(cx, 8 + y, 64), by = __shfl(cy, 8 + y, 64),
                      bz = __shfl(cz, 8 + y, 64), cb = __shfl(ch, 8 + y, 64);
            // octants of B's children: OR of 1 << octant over lanes 0 .. nb-1 (y = lane there)
            int bo = lane < nb ? 1 << (((bx & 1) << 2) | ((by & 1) << 1) | (bz & 1)) : 0;
            bo |= __shfl_xor(bo, 1, 64);
            bo |= __shfl_xor(bo, 2, 64);
            bo |= __shfl_xor(bo, 4, 64);
            bo = __shfl(bo, 0, 64);
            info[k] = (a0 != ga ? 1 : 0) | (b0 != gb ? 2 : 0) | ((((ax & 1) << 2) | ((ay & 1) << 1) | (az & 1)) << 10) |
                      (bo << 13);
            // a cell's pair with itself is always kept: it carries every leaf's self pair,
            // which the near-field lists rely on (at least one pair per leaf).  The lane's
            // cells are set whether or not the pair is kept: the slot's lead lane (y = 0)
            // names the target of the slot's kept pairs.
            const int ka = __shfl(kd, x, 64), kb = __shfl(kd, 8 + y, 64);
            if (x < na && y < nb) {
                pa[k] = a0 + x;
                pb[k] = b0 + y;
            }
            if (x < na && y < nb && (a0 + x == b0 + y || pair_carries(ka, kb))) {
                // rule 1, the MAC: accept A <- B iff A != B and theta |c_A - c_B| >= R_A + R_B
                // (R = half side), exactly: centres and radii in units of the finer half side
                const int lf = la > lb ? la : lb;
                const int64_t sa = int64_t(1) << (lf - la), sb = int64_t(1) << (lf - lb);
                const int64_t dx = (2 * (int64_t)bx + 1) * sb - (2 * (int64_t)ax + 1) * sa;
                const int64_t dy = (2 * (int64_t)by + 1) * sb - (2 * (int64_t)ay + 1) * sa;
                const int64_t dz = (2 * (int64_t)bz + 1) * sb - (2 * (int64_t)az + 1) * sa;
                const int64_t d2 = dx * dx + dy * dy + dz * dz, sr = sa + sb;
                if (pa[k] != pb[k] && theta2 * (double)d2 >= (double)(sr * sr)) {
                    act[k] = 0;
                    if (dx < -kKeyOffBias || dx >= kKeyOffBias || dy < -kKeyOffBias || dy >= kKeyOffBias ||
                        dz < -kKeyOffBias || dz >= kKeyOffBias)
                        o.flags[0] = 1;
                    else
                        key[k] = pack_key(lb - la, dx, dy, dz);
                } else {
                    act[k] = (ca == 0 && cb == 0) ? 1 : 2;   // rule 2, else rules 3-4 at the next step
                }
            }
        }
        const uint64_t bm = __ballot(act[k] == 0);
        cw[0] += __popcll(bm);
        cw[1] += __popcll(__ballot(act[k] == 1));
        cw[2] += __popcll(__ballot(act[k] == 2));
        cw[3] += __popcll(__ballot(y == 0 && ((bm >> (8 * x)) & 0xffull) != 0));
    }
    int off[4], tot[4];
    block_scan_waves4(cw, off, tot);
    __shared__ unsigned long long base[4];
    if (threadIdx.x < 4) base[threadIdx.x] = tot[threadIdx.x] ? atomicAdd(&cnt[threadIdx.x], (unsigned long long)tot[threadIdx.x]) : 0;
    __syncthreads();
    int64_t wm = (int64_t)base[0] + off[0], wq = (int64_t)base[1] + off[1], wn = (int64_t)base[2] + off[2],
            wr = (int64_t)base[3] + off[3];
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int k = 0; k < kTravPerWave; ++k) {
        const int2 v = make_int2(pa[k], pb[k]);
        const uint64_t bm = __ballot(act[k] == 0), bq = __ballot(act[k] == 1), bn = __ballot(act[k] == 2);
        const int mine = (int)((bm >> (8 * x)) & 0xffull);
        const bool lead = y == 0 && mine != 0;
        const uint64_t br = __ballot(lead);
        if (act[k] == 0) {
            const int64_t i = wm + __popcll(bm & lt);
            if (i < o.cap_m) {
                o.m2l[i] = v;
                o.m2l_slot[i] = key_slot(key[k], o.table, o.mask, o.flags);
            }
        } else if (act[k] == 1) {
            const int64_t i = wq + __popcll(bq & lt);
            if (i < o.cap_p) o.p2p[i] = v;
        } else if (act[k] == 2) {
            const int64_t i = wn + __popcll(bn & lt);
            if (i < o.cap_n) o.next[i] = v;
        }
        if (lead) {   // one lane per slot: the target is marked and the record written
            o.is_target[pa[k]] = 1;
            const int64_t i = wr + __popcll(br & lt);
            const int64_t first = wm + __popcll(bm & lt);   // lane 8x: the M2L pairs of lanes < 8x come first
            if (i < o.cap_r) o.rec[i] = make_int4(pa[k], (int)first, src0[k], info[k] | (mine << 2));
        }
        wm += __popcll(bm);
        wq += __popcll(bq);
        wn += __popcll(bn);
        wr += __popcll(br);
    }
}

// ----------------------------------------------------------------- M2L grouping

// Sum of one 64-bit value per thread over a 256-thread block, added once per block.
__device__ inline void block_add_u64(unsigned long long v, unsigned long long *dst) {
    __shared__ unsigned long long ws[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = ws[0] + ws[1] + ws[2] + ws[3];
        if (t) atomicAdd(dst, t);
    }
}

// Insert the key of every M2L pair into the table and record the pair's slot.  The
// traversal does this as it emits the pairs; this pass rebuilds a table that filled up
// there, at a larger size.
__global__ void k_key_insert(const int2 *pairs, int64_t np, CellView C, uint64_t *table, uint64_t mask,
                             int32_t *pair_slot, int32_t *flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x)
        pair_slot[i] = key_slot(pair_key(C, pairs[i].x, pairs[i].y, flags), table, mask, flags);
}

// Occupied slots of the key table, compacted for the host: out[0] = their number,
// out[1] = the table's flag word, out[2 + i] = the keys in no particular order (the
// first cap of them; the host sorts them).
__global__ void k_key_compact(const uint64_t *table, uint64_t H, uint64_t cap, unsigned long long *out) {
    for (uint64_t h = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; h < H; h += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t v = table[h];
        if (v != ~0ull) {
            const unsigned long long i = atomicAdd(&out[0], 1ull);
            if (i < cap) out[2 + i] = v;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[1] = table[H];
}

// Key id of every occupied slot: the rank of its key among the sorted distinct keys.
__global__ void k_slot_ids(const uint64_t *table, uint64_t H, const uint64_t *keys, int64_t nkeys, int32_t *slot_id) {
    for (uint64_t h = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; h < H; h += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t v = table[h];
        int32_t id = -1;
        if (v != ~0ull) {
            int64_t lo = 0, hi = nkeys;   // first index with keys[i] >= v
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (keys[mid] < v) lo = mid + 1;
                else hi = mid;
            }
            id = (int32_t)lo;
        }
        slot_id[h] = id;
    }
}

// Key id of every pair (from its slot), the (tile, key) table of target lanes (bit l: the
// target in lane l of the tile has a source under that key), and the number of pairs whose
// key joins cells of the same level.
// The lane masks are stored per tile in a row of `row` words, the key of id k at position
// lpos[oct * nkeys + k] for the tile's target octant oct: the keys of the pairs that one
// target has with the children of one split source cell sit together (eight positions,
// one 64-byte line), so that the lanes of one slot OR into a single line.
__global__ void __launch_bounds__(256) k_key_ids(const int2 *pairs, int64_t np, const int32_t *slot_id,
                                                 const int32_t *key_same, const int32_t *cell_tile,
                                                 const int32_t *cell_lane, const uint8_t *tile_oct,
                                                 const int32_t *lpos, int64_t nkeys, int64_t row,
                                                 int32_t *pair_key_id, unsigned long long *lanes,
                                                 unsigned long long *nsame) {
    static_assert(kTileN == 64, "one 64-bit lane mask per (tile, key)");
    unsigned long long loc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        const int id = slot_id[pair_key_id[i]];
        pair_key_id[i] = id;
        const int a = pairs[i].x, t = cell_tile[a];
        atomicOr(&lanes[(int64_t)t * row + lpos[(int64_t)tile_oct[t] * nkeys + id]], 1ull << cell_lane[a]);
        loc += key_same[id] ? 1ull : 0ull;
    }
    block_add_u64(loc, nsame);
}

// A (tile, key) cell becomes an entry of the target tile (dense) when its sources fill at
// least fill_pct percent of the 16-column blocks it touches, or when the tile is one of the
// first `all_dense` tiles; its pairs go to the slot pool otherwise.
__global__ void __launch_bounds__(256) k_dense_flags(const unsigned long long *lanes, const uint8_t *tile_oct,
                                                     const int32_t *lpos, int64_t row, int64_t ntk, int64_t nkeys,
                                                     int fill_pct, int64_t all_dense, int32_t *present,
                                                     unsigned long long *sparse_pairs) {
    unsigned long long loc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntk; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / nkeys;
        const unsigned long long m = lanes[t * row + lpos[(int64_t)tile_oct[t] * nkeys + i % nkeys]];
        int f = 0;
        if (m) {
            int blocks = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) blocks += ((m >> (16 * b)) & 0xffffull) != 0;
            f = (i / nkeys < all_dense || 100 * __popcll(m) >= fill_pct * 16 * blocks) ? 1 : 0;
            if (!f) loc += (unsigned long long)__popcll(m);
        }
        present[i] = f;
    }
    if (sparse_pairs) block_add_u64(loc, sparse_pairs);
}

// Entries are the dense (tile, key) cells in tile-major, key-ascending order; the pairs of
// the other cells are flagged for the slot pool (when `pool` is given).
// `entry_of` is the exclusive scan of the dense flags with the total appended, so a cell
// is dense iff its successor's value is larger.
__global__ void k_fill_entries(const int2 *pairs, int64_t np, const int32_t *pair_key_id, const int32_t *cell_tile,
                               const int32_t *cell_lane, const int32_t *entry_of, int64_t nkeys, int32_t *entry_src,
                               uint8_t *pool) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        const int2 pr = pairs[i];
        const int64_t tk = (int64_t)cell_tile[pr.x] * nkeys + pair_key_id[i];
        const int e = entry_of[tk];
        const bool dense = entry_of[tk + 1] > e;
        if (pool) pool[i] = dense ? 0 : 1;
        if (dense) entry_src[(int64_t)e * kTileN + cell_lane[pr.x]] = pr.y;
    }
}

// ---------------------------------------------------------------- M2L slot pool
// Pairs of sparse (tile, key) cells are regrouped by the pair of cells the traversal split
// to produce them: a slot is (target t, the source-side cell B of that pair), holding the
// pairs (t, child of B) -- or the one pair (t, B) when B was not split.  The traversal
// writes the pairs of a slot consecutively, in source order, with one record per slot.
// Slots whose pooled pairs have the same key sequence (signature) share tiles of 64
// columns, one column per slot, so every column of every entry holds a source; each
// slot's column is a partial local expansion of its target, and the targets' partials are
// summed in a fixed order.

// Position of the n-th lowest set bit of v (n < popcount(v)).
__device__ inline int nth_bit(unsigned v, int n) {
    for (; n > 0; --n) v &= v - 1;
    return __builtin_ctz(v);
}

// Pooled pairs of every slot record (bit j: the record's j-th pair went to the pool);
// records with any are flagged.
__global__ void k_rec_members(const int4 *rec, int64_t nrec, const uint8_t *pool, int32_t *mbits, int32_t *flag) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrec; r += (int64_t)gridDim.x * blockDim.x) {
        const int4 R = rec[r];
        const int c = __popc((R.w >> 2) & 0xff);
        int m = 0;
        for (int j = 0; j < c; ++j) m |= pool[(int64_t)R.y + j] ? 1 << j : 0;
        mbits[r] = m;
        flag[r] = m != 0;
    }
}

// Sort keys of the pooled slots: (target, key id of the slot's first pooled pair) in
// `kbits` + the target's bits.  Unique per slot -- a pair (target, source) is in exactly one
// slot, and a target and an operator key fix the source cell -- so the order is the same on
// every run whatever order the traversal wrote the records in; values = record index.
__global__ void k_rec_keys(const int4 *rec, const int32_t *flag, const int32_t *at, const int32_t *mbits,
                           const int32_t *key_id, int64_t nrec, int kbits, uint64_t *keys, int32_t *vals) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrec; r += (int64_t)gridDim.x * blockDim.x)
        if (flag[r]) {
            const int4 R = rec[r];
            const int64_t j = at[r];
            keys[j] = ((uint64_t)R.x << kbits) | (uint64_t)(uint32_t)key_id[(int64_t)R.y + __builtin_ctz(mbits[r])];
            vals[j] = (int32_t)r;
        }
}

// Per slot (in sorted order): first pair of its record and its pooled pairs (bits relative
// to the first), b0 and the source mask of its pooled pairs, target, and signature = (key
// id of its first pooled pair, target side split, source side split, target octant when
// split, octants of its pooled sources when split).  Given how the producing pair was
// split, the first key, the target octant and the source octants fix that pair's geometry
// and so every key of the slot in source order: slots with equal signatures have equal
// key sequences.
__global__ void __launch_bounds__(256) k_slot_info(const int4 *rec, const int32_t *mbits, const int32_t *order,
                                                   int64_t ns, const int32_t *key_id, int32_t *slot_first,
                                                   int32_t *slot_mb, int32_t *slot_b0, int32_t *slot_ym,
                                                   int32_t *slot_tgt, uint64_t *slot_sig,
                                                   unsigned long long *partial_octants) {
    unsigned long long part = 0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ns; q += (int64_t)gridDim.x * blockDim.x) {
        const int r = order[q];
        const int4 R = rec[r];
        const int m = mbits[r], g = R.w & 3, ym = (R.w >> 2) & 0xff, bo = (R.w >> 13) & 0xff;
        int pym = 0, smask = 0;
        for (int mm = m; mm; mm &= mm - 1) {
            const int y = nth_bit((unsigned)ym, __builtin_ctz(mm));
            pym |= 1 << y;
            if (g & 2) smask |= 1 << nth_bit((unsigned)bo, y);
        }
        if ((g & 2) && __popc(m) < 8) ++part;
        const uint64_t ot = (g & 1) ? (uint64_t)((R.w >> 10) & 7) : 0;
        slot_first[q] = R.y;
        slot_mb[q] = m;
        slot_b0[q] = R.z;
        slot_ym[q] = pym;
        slot_tgt[q] = R.x;
        slot_sig[q] = (uint64_t)(uint32_t)key_id[(int64_t)R.y + __builtin_ctz(m)] | ((uint64_t)(g & 1) << 32) |
                      ((uint64_t)((g >> 1) & 1) << 33) | (ot << 34) | ((uint64_t)smask << 37);
    }
    block_add_u64(part, partial_octants);
}

// Signature table: every slot's signature inserted (its table slot recorded).  Probing
// stops after kSigProbes slots and flags the table as full, so that a table too small for
// the signatures costs one bounded pass before it is rebuilt larger.
constexpr int kSigProbes = 64;
__global__ void k_sig_insert(const uint64_t *sig, int64_t ns, uint64_t *table, uint64_t mask, int32_t *at,
                             int32_t *flags) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ns; q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = sig[q];
        uint64_t h = key_hash(key) & mask;
        int32_t got = -1;
        for (int probe = 0; probe < kSigProbes; ++probe) {
            const uint64_t cur = table[h];
            if (cur == key) { got = (int32_t)h; break; }
            if (cur == kEmpty) {
                const uint64_t prev = atomicCAS((unsigned long long *)&table[h], (unsigned long long)kEmpty,
                                                (unsigned long long)key);
                if (prev == kEmpty || prev == key) { got = (int32_t)h; break; }
            }
            h = (h + 1) & mask;
        }
        if (got < 0) {
            flags[1] = 1;
            got = 0;
        }
        at[q] = got;
    }
}

// Signature id of every slot.
__global__ void k_sig_ids(const int32_t *at, const int32_t *table_id, int64_t ns, int32_t *sig_id) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ns; q += (int64_t)gridDim.x * blockDim.x)
        sig_id[q] = table_id[at[q]];
}
// One representative slot per signature: the first slot of one of its groups (any slot of a
// signature has the signature's key sequence).
__global__ void k_group_rep(const int32_t *gflag, const int32_t *sorted, const int32_t *sig_id, int64_t ns,
                            int32_t *rep) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ns; j += (int64_t)gridDim.x * blockDim.x)
        if (gflag[j]) rep[sig_id[sorted[j]]] = sorted[j];
}

// Key sequence of every signature, from its representative slot ([nsig][8], count in sig_n).
__global__ void k_sig_keys(const int32_t *rep, int64_t nsig, const int32_t *slot_first, const int32_t *slot_mb,
                           const int32_t *key_id, int32_t *sig_keys, int32_t *sig_n) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < nsig; g += (int64_t)gridDim.x * blockDim.x) {
        const int q = rep[g], f = slot_first[q];
        int e = 0;
        for (int mm = slot_mb[q]; mm; mm &= mm - 1) sig_keys[g * 8 + e++] = key_id[(int64_t)f + __builtin_ctz(mm)];
        sig_n[g] = e;
        for (; e < 8; ++e) sig_keys[g * 8 + e] = 0;
    }
}

// Tile order of the slots: (region of the target, signature, target).  The region is the
// target's ancestor (or, for a coarser target, its descendant corner) at level `rl`, so the
// workgroups in flight share operators (one signature) and source expansions (one region).
// The slots are numbered in target order and the radix sort is stable, so the sort key
// needs only (region, signature).
__global__ void k_slot_sort_keys(const int32_t *slot_tgt, const int32_t *sig_id, int64_t ns, CellView C, int rl,
                                 int sbits, uint64_t *keys, int32_t *vals) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ns; q += (int64_t)gridDim.x * blockDim.x) {
        const int t = slot_tgt[q], l = C.level[t];
        const uint64_t pre = C.prefix[t];
        const uint64_t reg = l >= rl ? pre >> (3 * (l - rl)) : pre << (3 * (rl - l));
        keys[q] = (reg << sbits) | (uint64_t)sig_id[q];
        vals[q] = (int32_t)q;
    }
}

// Group starts along the sorted slots: (region, signature) changes.
__global__ void k_group_flags(const uint64_t *keys, int64_t ns, int32_t *flag) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ns; j += (int64_t)gridDim.x * blockDim.x)
        flag[j] = (j == 0 || keys[j] != keys[j - 1]) ? 1 : 0;
}
__global__ void k_group_starts(const int32_t *flag, const int32_t *gid, int64_t ns, int32_t *gstart) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ns; j += (int64_t)gridDim.x * blockDim.x)
        if (flag[j]) gstart[gid[j]] = (int32_t)j;
}
// A tile starts at every 64th slot of a group.
__global__ void k_tile_flags(const int32_t *flag, const int32_t *gid, const int32_t *gstart, int64_t ns,
                             int32_t *tflag) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ns; j += (int64_t)gridDim.x * blockDim.x) {
        const int g = gid[j] + flag[j] - 1;
        tflag[j] = ((j - gstart[g]) % kTileN) == 0 ? 1 : 0;
    }
}
// Per slot tile: its signature and number of entries.
__global__ void k_tile_sig(const int32_t *tflag, const int32_t *tid, const int32_t *sorted, const int32_t *sig_id,
                           const int32_t *sig_n, int64_t ns, int32_t *tile_sig, int32_t *tile_ne) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ns; j += (int64_t)gridDim.x * blockDim.x)
        if (tflag[j]) {
            const int T = tid[j], g = sig_id[sorted[j]];
            tile_sig[T] = g;
            tile_ne[T] = sig_n[g];
        }
}
// Entries of the slot tiles (keys, sources per column) and each slot's partial column:
// slot tile T is partial tile `part0 + T`.
__global__ void k_slot_entries(const int32_t *tflag, const int32_t *tid, const int32_t *flag, const int32_t *gid,
                               const int32_t *gstart, const int32_t *sorted, int64_t ns, const int32_t *slot_b0,
                               const int32_t *slot_ym, const int32_t *tile_eoff, int64_t e_base, int64_t part0,
                               int32_t *entry_src, int64_t *slot_pos) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ns; j += (int64_t)gridDim.x * blockDim.x) {
        const int T = tid[j] + tflag[j] - 1;
        const int lane = (int)((j - gstart[gid[j] + flag[j] - 1]) % kTileN);
        const int q = sorted[j], b0 = slot_b0[q];
        int64_t e = e_base + tile_eoff[T];
        for (int ym = slot_ym[q]; ym; ym &= ym - 1, ++e) entry_src[e * kTileN + lane] = b0 + __builtin_ctz(ym);
        slot_pos[q] = (part0 + T) * kTileN + lane;
    }
}
__global__ void k_slot_entry_keys(const int32_t *tile_sig, const int32_t *tile_eoff, int64_t nt,
                                  const int32_t *sig_keys, const int32_t *sig_n, int64_t e_base, int32_t *entry_key) {
    for (int64_t T = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; T < nt; T += (int64_t)gridDim.x * blockDim.x) {
        const int g = tile_sig[T];
        for (int e = 0; e < sig_n[g]; ++e) entry_key[e_base + tile_eoff[T] + e] = sig_keys[g * 8 + e];
    }
}
// Work items of the slot tiles, after the dense ones: every slot tile writes its partial.
__global__ void k_slot_work(const int32_t *tile_eoff, const int32_t *tile_ne, int64_t nt, int64_t e_base,
                            int64_t part0, int4 *work) {
    for (int64_t T = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; T < nt; T += (int64_t)gridDim.x * blockDim.x) {
        const int e0 = (int)(e_base + tile_eoff[T]);
        work[T] = make_int4(0, e0, e0 + tile_ne[T], (int)(part0 + T + 1));
    }
}
// Runs of slots with one target (slots are numbered in target order).
__global__ void k_run_flags(const int32_t *slot_tgt, int64_t ns, int32_t *flag) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ns; q += (int64_t)gridDim.x * blockDim.x)
        flag[q] = (q == 0 || slot_tgt[q] != slot_tgt[q - 1]) ? 1 : 0;
}
__global__ void k_shift_pos(int64_t *pos, int64_t n, int64_t by) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pos[i] += by;
}
__global__ void k_run_info(const int32_t *flag, const int32_t *rid, const int32_t *slot_tgt, int64_t ns,
                           int32_t *run_first, int32_t *run_tgt) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ns; q += (int64_t)gridDim.x * blockDim.x)
        if (flag[q]) {
            run_first[rid[q]] = (int32_t)q;
            run_tgt[rid[q]] = slot_tgt[q];
        }
}

__global__ void k_entry_keys(const int32_t *present, const int32_t *entry_of, int64_t ntk, int64_t nkeys,
                             int32_t *entry_key) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntk; i += (int64_t)gridDim.x * blockDim.x)
        if (present[i]) entry_key[entry_of[i]] = (int32_t)(i % nkeys);
}

// Column-block mask of every entry: bit cb set iff one of its columns 16cb..16cb+15 has a
// source; optionally the entry's number of sources.
__global__ void k_entry_masks(const int32_t *entry_src, int64_t ne, uint8_t *m8, int32_t *nsrc) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int4 *row = reinterpret_cast<const int4 *>(entry_src + e * kTileN);
        int m = 0, c = 0;
        for (int q = 0; q < kTileN / 4; ++q) {
            const int4 v = row[q];
            if (v.x >= 0 || v.y >= 0 || v.z >= 0 || v.w >= 0) m |= 1 << (q / 4);
            c += (v.x >= 0) + (v.y >= 0) + (v.z >= 0) + (v.w >= 0);
        }
        m8[e] = (uint8_t)m;
        if (nsrc) nsrc[e] = c;
    }
}

__global__ void k_tile_first(const int32_t *entry_of, int64_t ntiles, int64_t nkeys, int32_t *tile_first) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x)
        tile_first[t] = entry_of[t * nkeys];
}


// Boundary class of a cell: per axis, its distance (in cells of its octant, capped at 2)
// to the low and to the high face of the root cube, 9 values per axis.  Cells of one
// class and octant have the same interaction offsets in a uniform region, so ordering a
// tile's targets by class first fills the MFMA column blocks of an M2L entry better.
constexpr int kClassBits = 10;   // 9^3 = 729 classes
__device__ inline int boundary_class(const CellView &C, int c) {
    const int l = C.level[c];
    if (l == 0) return 0;
    const int nl = 1 << (l - 1);   // cells of one octant per axis
    auto axis = [&](int v) {
        v >>= 1;
        return min(v, 2) * 3 + min(nl - 1 - v, 2);
    };
    return (axis(C.ix[c]) * 9 + axis(C.iy[c])) * 9 + axis(C.iz[c]);
}

// Sort key of a tile target: (level, octant) bucket above `cls_bits` bits of boundary
// class (0 or kClassBits); equal keys keep the cell (Morton) order.
__global__ void k_target_keys(const int32_t *is_target, const int32_t *ex, int64_t nc, CellView C, int by_octant,
                              int cls_bits, uint64_t *tkeys, int32_t *tvals) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        if (!is_target[c]) continue;
        int oct = by_octant ? ((C.ix[c] & 1) << 2) | ((C.iy[c] & 1) << 1) | (C.iz[c] & 1) : 0;
        uint64_t k = (uint64_t)(C.level[c] * 8 + oct) << cls_bits;
        if (cls_bits) k |= (uint64_t)boundary_class(C, (int)c);
        tkeys[ex[c]] = k;
        tvals[ex[c]] = (int32_t)c;
    }
}

__global__ void k_bucket_starts(const uint64_t *tkeys, int64_t nt, int cls_bits, int32_t *bstart) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nt; i += (int64_t)gridDim.x * blockDim.x) {
        int b = (int)(tkeys[i] >> cls_bits);
        if (i == 0 || (int)(tkeys[i - 1] >> cls_bits) != b) bstart[b] = (int32_t)i;
    }
}

constexpr int kBuckets = (kMaxLevel + 1) * 8;
constexpr int64_t kGroupedKeysMax = 8192;   // the grouped lane-mask layout up to this many keys
struct BucketBase {   // first tile of every (level, octant) bucket, passed by value
    int32_t v[kBuckets];
};
__global__ void k_assign_tiles(const uint64_t *tkeys, const int32_t *tvals, int64_t nt, int cls_bits,
                               const int32_t *bstart, BucketBase tbase, int32_t *cell_tile, int32_t *cell_lane,
                               int32_t *tile_targets) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nt; i += (int64_t)gridDim.x * blockDim.x) {
        int b = (int)(tkeys[i] >> cls_bits);
        int r = (int)(i - bstart[b]);
        int tile = tbase.v[b] + r / kTileN, lane = r % kTileN;
        int c = tvals[i];
        cell_tile[c] = tile;
        cell_lane[c] = lane;
        tile_targets[(int64_t)tile * kTileN + lane] = c;
    }
}



// ----------------------------------------------------------------- M2M / L2L tiles
__global__ void k_flag_internal(const int32_t *nchild, int64_t nc, int32_t *flag) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x)
        flag[c] = nchild[c] > 0 ? 1 : 0;
}
__global__ void k_flag_nonroot(const int32_t *level, int64_t nc, int32_t *flag) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x)
        flag[c] = level[c] > 0 ? 1 : 0;
}
// M2M: target = parent cell, one entry per child octant, source = the child in that octant.
__global__ void k_m2m_entries(int64_t nc, CellView C, const int32_t *cell_tile, const int32_t *cell_lane,
                              int32_t *entry_src) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        int nch = C.nchild[c];
        if (nch == 0) continue;
        int t = cell_tile[c], lane = cell_lane[c];
        for (int q = 0; q < nch; ++q) {
            int ch = C.child0[c] + q;
            int oct = ((C.ix[ch] & 1) << 2) | ((C.iy[ch] & 1) << 1) | (C.iz[ch] & 1);
            entry_src[((int64_t)t * 8 + oct) * kTileN + lane] = ch;
        }
    }
}
// L2L: target = cell, one entry per tile (all targets of a tile share the octant), source = parent.
__global__ void k_l2l_entries(int64_t nc, CellView C, const int32_t *parent, const int32_t *cell_tile,
                              const int32_t *cell_lane, int32_t *entry_key, int32_t *entry_src) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        if (C.level[c] == 0) continue;
        int t = cell_tile[c], lane = cell_lane[c];
        entry_src[(int64_t)t * kTileN + lane] = parent[c];
        if (lane == 0) entry_key[t] = ((C.ix[c] & 1) << 2) | ((C.iy[c] & 1) << 1) | (C.iz[c] & 1);
    }
}
__global__ void k_work_uniform(int64_t ntiles, int per, int32_t *entry_key_mod8, int4 *work) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) {
        work[t] = make_int4((int)t, (int)(t * per), (int)(t * per + per), 0);
        if (entry_key_mod8)
            for (int q = 0; q < per; ++q) entry_key_mod8[t * per + q] = q;
    }
}

// ----------------------------------------------------------------- P2P lists
__global__ void k_leaf_flags(const int32_t *nchild, int64_t nc, int32_t *flag) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x)
        flag[c] = nchild[c] == 0 ? 1 : 0;
}
__global__ void k_leaf_compact(const int32_t *flag, const int32_t *ex, int64_t nc, int32_t *leaves, int32_t *leaf_id) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        leaf_id[c] = flag[c] ? ex[c] : -1;
        if (flag[c]) leaves[ex[c]] = (int32_t)c;
    }
}

// Leaf cell of every body (sorted order): the leaves' body ranges partition the bodies.
__global__ void k_body_leaf(const int32_t *leaves, int64_t nleaves, const int32_t *c_start, const int32_t *c_count,
                            int32_t *body_leaf) {
    for (int64_t li = blockIdx.x; li < nleaves; li += gridDim.x) {
        const int c = leaves[li], s0 = c_start[c], cnt = c_count[c];
        for (int j = threadIdx.x; j < cnt; j += blockDim.x) body_leaf[s0 + j] = c;
    }
}

// (target leaf id, source leaf id) packed into `lbits`-bit halves; the value is the source cell.
__global__ void k_p2p_composite(const int2 *pairs, int64_t np, const int32_t *leaf_id, int lbits, uint64_t *comp,
                                int32_t *vals) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        comp[i] = ((uint64_t)leaf_id[pairs[i].x] << lbits) | (uint64_t)leaf_id[pairs[i].y];
        vals[i] = pairs[i].y;
    }
}

__global__ void __launch_bounds__(256) k_p2p_csr(const uint64_t *comp, const int32_t *src, int64_t np, int lbits,
                                                 const int32_t *leaves, int2 *pairs_out, int32_t *pair_off,
                                                 const int32_t *c_count, unsigned long long *inter) {
    unsigned long long loc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        int la = (int)(comp[i] >> lbits);
        int a = leaves[la], b = src[i];
        pairs_out[i] = make_int2(a, b);
        if (i == 0 || (int)(comp[i - 1] >> lbits) != la) pair_off[la] = (int32_t)i;
        unsigned long long ca = (unsigned long long)c_count[a], cb = (unsigned long long)c_count[b];
        loc += (a == b) ? ca * (ca - 1) : ca * cb;
    }
    block_add_u64(loc, inter);
}

// Source runs of each target leaf: its source leaves (self excluded), in Morton order,
// with adjacent body ranges merged into one run.  Built in parallel over pairs (pairs are
// sorted by (target, source), so a target's sources are consecutive): a pair opens a run
// unless the previous non-self pair of the same target ends where this one starts.
__device__ inline int64_t p2p_prev(const int2 *pairs, int64_t k, int a) {   // previous non-self pair of target a
    int64_t j = k - 1;
    if (j >= 0 && pairs[j].x == a && pairs[j].y == a) --j;
    return (j >= 0 && pairs[j].x == a) ? j : -1;
}
__device__ inline int64_t p2p_next(const int2 *pairs, int64_t k, int64_t np, int a) {
    int64_t j = k + 1;
    if (j < np && pairs[j].x == a && pairs[j].y == a) ++j;
    return (j < np && pairs[j].x == a) ? j : -1;
}

__global__ void k_p2p_run_flags(const int2 *pairs, int64_t np, const int32_t *c_start, const int32_t *c_count,
                                int32_t *open) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < np; k += (int64_t)gridDim.x * blockDim.x) {
        const int a = pairs[k].x, b = pairs[k].y;
        int f = 0;
        if (a != b) {
            const int64_t j = p2p_prev(pairs, k, a);
            f = (j < 0 || c_start[pairs[j].y] + c_count[pairs[j].y] != c_start[b]) ? 1 : 0;
        }
        open[k] = f;
    }
}

// A run's first pair writes its start, its last pair its end; run ids come from the
// exclusive scan of the open flags.  seg_off[li] is the run id at the leaf's first pair.
__global__ void k_p2p_run_write(const int2 *pairs, int64_t np, const int32_t *c_start, const int32_t *c_count,
                                const int32_t *open, const int32_t *run_id, int2 *segs) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < np; k += (int64_t)gridDim.x * blockDim.x) {
        const int a = pairs[k].x, b = pairs[k].y;
        if (a == b) continue;
        const int id = run_id[k] + open[k] - 1;
        if (open[k]) segs[id].x = c_start[b];
        const int64_t j = p2p_next(pairs, k, np, a);
        if (j < 0 || open[j]) segs[id].y = c_start[b] + c_count[b];   // end for now; length below
    }
}

__global__ void k_p2p_run_len(int2 *segs, const int64_t *nseg_dev) {
    const int64_t nseg = *nseg_dev;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nseg; i += (int64_t)gridDim.x * blockDim.x) {
        int2 r = segs[i];
        segs[i] = make_int2(r.x, r.y - r.x);
    }
}

__global__ void k_p2p_seg_off(int64_t nl, const int32_t *pair_off, const int32_t *run_id, const int64_t *nseg,
                              int32_t *seg_off) {
    for (int64_t li = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; li <= nl; li += (int64_t)gridDim.x * blockDim.x)
        seg_off[li] = li < nl ? run_id[pair_off[li]] : (int32_t)*nseg;
}

// Near-field work items: a target leaf whose list holds more than kP2PPieceWork
// interactions (and at most kP2PThreads targets) is cut into pieces of about equal source
// counts; lens[r] is the length of run r (0 past the last run).
__global__ void k_p2p_run_len64(const int2 *segs, const int64_t *nseg, int64_t n, int64_t *lens) {
    const int64_t ns = *nseg;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        lens[r] = r < ns ? (int64_t)segs[r].y : 0;
}
__global__ void k_p2p_split(int64_t nl, const int32_t *leaves, const int32_t *c_count, const int32_t *seg_off,
                            const int64_t *run_pre, int32_t *pieces, int32_t *part_len) {
    for (int64_t li = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; li < nl; li += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tn = c_count[leaves[li]];
        const int64_t S = run_pre[seg_off[li + 1]] - run_pre[seg_off[li]];
        int64_t k = 1;
        if (tn <= kP2PThreads && tn * S > kP2PPieceWork)
            k = std::min<int64_t>(std::min<int64_t>(kP2PMaxPieces, S), (tn * S + kP2PPieceWork - 1) / kP2PPieceWork);
        pieces[li] = (int32_t)k;
        part_len[li] = k > 1 ? (int32_t)k : 0;
    }
}
__global__ void k_p2p_items(int64_t nl, const int32_t *pieces, const int32_t *item_off, const int32_t *part_off,
                            int4 *items) {
    for (int64_t li = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; li < nl; li += (int64_t)gridDim.x * blockDim.x) {
        const int k = pieces[li], o = item_off[li], pb = k > 1 ? part_off[li] : -1;
        for (int j = 0; j < k; ++j) items[o + j] = make_int4((int)li, j, k, pb);
    }
}

// ----------------------------------------------------------------- host side
static int grid1(int64_t n, int bs = 256) {
    int64_t g = (n + bs - 1) / bs;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}
static int bits_for(int64_t v) {   // number of bits to hold values in [0, v)
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return std::max(b, 1);
}

template <class T>
static void grow(Alloc &a, T *&buf, int64_t &cap, int64_t used, int64_t need, hipStream_t s) {
    if (need <= cap) return;
    int64_t nc = std::max<int64_t>(need, cap * 2);
    T *nb = a.get_n<T>(nc);
    if (used > 0) HIP_CHECK(hipMemcpyAsync(nb, buf, sizeof(T) * used, hipMemcpyDeviceToDevice, s));
    if (buf) a.put(buf);
    buf = nb;
    cap = nc;
}

// Tiles of kTileN cells: the flagged cells grouped by level (and octant when
// by_octant), inside a group by boundary class (when by_class) and then in Morton order.
// Returns the number of tiles; fills tile_targets ([ntiles][kTileN], -1 = empty lane),
// cell -> (tile, lane) maps and the first tile of every (level, octant) bucket (host,
// size kBuckets + 1).
static int64_t tile_cells(const CellView &C, int64_t nc, int32_t *flag, bool by_octant, bool by_class, Alloc &a,
                          hipStream_t s, int32_t *&tile_targets, int32_t *cell_tile, int32_t *cell_lane,
                          std::vector<int32_t> &bucket_tile, int64_t &ntargets) {
    const int cls_bits = by_class ? kClassBits : 0;
    int32_t *tex = a.get_n<int32_t>(nc);
    int64_t nt = exclusive_scan_i32(flag, tex, nc, a, s);
    ntargets = nt;
    bucket_tile.assign(kBuckets + 1, 0);
    if (nt == 0) {
        a.put(tex);
        tile_targets = a.get_n<int32_t>(1);
        return 0;
    }
    uint64_t *tk = a.get_n<uint64_t>(nt);
    int32_t *tv = a.get_n<int32_t>(nt);
    hipLaunchKernelGGL(k_target_keys, grid1(nc), 256, 0, s, (const int32_t *)flag, (const int32_t *)tex, nc, C,
                       by_octant ? 1 : 0, cls_bits, tk, tv);
    static_assert(kBuckets <= 256, "buckets fit 8 bits");
    radix_sort_u64(tk, tv, nt, 8 + cls_bits, a, s);   // stable: Morton (= index) order among equal keys
    int32_t *bst = a.get_n<int32_t>(kBuckets);
    fill_i32(bst, -1, kBuckets, s);
    hipLaunchKernelGGL(k_bucket_starts, grid1(nt), 256, 0, s, (const uint64_t *)tk, nt, cls_bits, bst);
    std::vector<int32_t> hb_start(kBuckets);
    BucketBase hb_base{};
    {
        Mailbox &mb = *a.mb;
        const uint64_t t = mb.next_ticket();
        publish(bst, 4 * kBuckets, mb, t, s);
        mb.wait(t, s);
        std::memcpy(hb_start.data(), mb.data_host<int32_t>(), 4 * kBuckets);
    }
    int64_t ntiles = 0;
    for (int b = 0; b < kBuckets; ++b) {
        hb_base.v[b] = (int32_t)ntiles;
        bucket_tile[b] = (int32_t)ntiles;
        if (hb_start[b] < 0) continue;
        int64_t end = nt;
        for (int b2 = b + 1; b2 < kBuckets; ++b2)
            if (hb_start[b2] >= 0) { end = hb_start[b2]; break; }
        ntiles += (end - hb_start[b] + kTileN - 1) / kTileN;
    }
    bucket_tile[kBuckets] = (int32_t)ntiles;
    tile_targets = a.get_n<int32_t>(ntiles * kTileN);
    fill_i32(tile_targets, -1, ntiles * kTileN, s);
    hipLaunchKernelGGL(k_assign_tiles, grid1(nt), 256, 0, s, (const uint64_t *)tk, (const int32_t *)tv, nt, cls_bits,
                       (const int32_t *)bst, hb_base, cell_tile, cell_lane, tile_targets);
    a.put(tex); a.put(tk); a.put(tv); a.put(bst);
    return ntiles;
}

// Host-side stage timer, printed to stderr when FMM_LOG is set.
struct StageLog {
    bool on = getenv("FMM_LOG") != nullptr;
    hipStream_t s = nullptr;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now(), last = t0;
    void operator()(const char *what) {
        if (!on) return;
        (void)hipStreamSynchronize(s);   // attribute device time to the stage that queued it
        auto now = std::chrono::steady_clock::now();
        fprintf(stderr, "[fmm plan] %-28s +%8.3f ms  (t=%8.3f ms)\n", what,
                std::chrono::duration<double, std::milli>(now - last).count(),
                std::chrono::duration<double, std::milli>(now - t0).count());
        last = now;
    }
};

// Slot tiles of the M2L pool (see the slot pool kernels).  Device arrays of the plan's
// allocator; release() returns the temporaries.
constexpr int kDenseFillPct = 75;   // a (tile, key) cell stays a dense entry at >= 75% block fill
constexpr int kSlotRegionLevel = 1; // slot tiles are ordered by the targets' ancestor at this level
constexpr int kPoolMinPct = 5;      // a pool holding fewer than 5% of the M2L pairs is not built
constexpr int kSlotsPerSig = 64;    // fewer slots per signature on average: the pool is given up
struct SlotTiles {
    bool abandoned = false;                         // the pool's slots were too diverse to tile well
    int64_t nslots = 0, ntiles = 0, ne = 0, nsig = 0;
    int32_t *slot_first = nullptr, *slot_mb = nullptr, *slot_tgt = nullptr;   // slots in (target, first key) order
    int32_t *slot_b0 = nullptr, *slot_ym = nullptr;
    int32_t *sorted = nullptr;                      // tile order -> slot
    int32_t *gflag = nullptr, *gid = nullptr, *gstart = nullptr, *tflag = nullptr, *tid = nullptr;
    int32_t *tile_sig = nullptr, *tile_ne = nullptr, *tile_eoff = nullptr;
    int32_t *sig_keys = nullptr, *sig_n = nullptr;
    void release(Alloc &a) {
        for (int32_t *p : {slot_first, slot_mb, slot_tgt, slot_b0, slot_ym, sorted, gflag, gid, gstart, tflag, tid,
                           tile_sig, tile_ne, tile_eoff, sig_keys, sig_n})
            if (p) a.put(p);
        *this = SlotTiles{};
    }
};

// Groups the pool pairs into slots and slot tiles; fills P->slot_pos (partial column of
// every slot, relative to the first slot tile), P->run_first / P->run_tgt / P->nruns (the
// slots of each target, for the fixed-order sum) and `st` (what the entry builders need).
// Unless `keep`, gives the pool up (st.abandoned, no tiles) when its slots would tile poorly.
static void build_slots(fmm_plan_s *P, const CellView &C, const int32_t *key_id, const int4 *recs,
                        int64_t nrec, const uint8_t *pool, int64_t npool, Alloc &a, hipStream_t s, SlotTiles &st,
                        bool keep) {
    Mailbox &mb = *a.mb;
    StageLog lg;
    lg.s = s;
    const int64_t nc = P->ncells;
    const int cbits = bits_for(nc);
    // records with pooled pairs, sorted by (target, key of the first pooled pair)
    int32_t *mbits = a.get_n<int32_t>(nrec), *pflag = a.get_n<int32_t>(nrec), *pat = a.get_n<int32_t>(nrec);
    hipLaunchKernelGGL(k_rec_members, grid1(nrec), 256, 0, s, recs, nrec, pool, mbits, pflag);
    const int64_t ns = exclusive_scan_i32(pflag, pat, nrec, a, s);
    uint64_t *pk = a.get_n<uint64_t>(ns);
    int32_t *order = a.get_n<int32_t>(ns);
    const int kbits = bits_for(P->nkeys);
    hipLaunchKernelGGL(k_rec_keys, grid1(nrec), 256, 0, s, recs, (const int32_t *)pflag, (const int32_t *)pat,
                       (const int32_t *)mbits, key_id, nrec, kbits, pk, order);
    a.put(pflag); a.put(pat);
    radix_sort_u64(pk, order, ns, cbits + kbits, a, s);
    a.put(pk);
    lg("  slots: sort");
    st.nslots = ns;
    st.slot_first = a.get_n<int32_t>(ns);
    st.slot_mb = a.get_n<int32_t>(ns);
    st.slot_tgt = a.get_n<int32_t>(ns);
    st.slot_b0 = a.get_n<int32_t>(ns);
    st.slot_ym = a.get_n<int32_t>(ns);
    uint64_t *sig = a.get_n<uint64_t>(ns);
    unsigned long long *err = a.get_n<unsigned long long>(1);   // slots whose split source has empty octants
    fill_i32(reinterpret_cast<int32_t *>(err), 0, 2, s);
    hipLaunchKernelGGL(k_slot_info, std::min(grid1(ns), 8192), 256, 0, s, recs, (const int32_t *)mbits,
                       (const int32_t *)order, ns, key_id, st.slot_first, st.slot_mb, st.slot_b0, st.slot_ym,
                       st.slot_tgt, sig, err);
    a.put(mbits); a.put(order);
    int64_t partial_oct = 0;
    {
        const uint64_t t = mb.next_ticket();
        publish(err, 8, mb, t, s);
        mb.wait(t, s);
        partial_oct = (int64_t)mb.data_host<uint64_t>()[0];
    }
    lg("  slots: slot info");
    if (lg.on) fprintf(stderr, "[fmm plan]   %lld of %lld slots from sources with empty octants\n",
                       (long long)partial_oct, (long long)ns);
    if (!keep && 2 * partial_oct > ns) {
        // most sources miss octants (a surface-like cloud): signatures would be too many
        a.put(sig); a.put(err);
        st.release(a);
        st.abandoned = true;
        lg("  slots: given up (sources with empty octants)");
        return;
    }

    // distinct signatures through a device hash table (rebuilt larger while more than half full)
    uint64_t H = uint64_t(1) << 16;
    int32_t *at = a.get_n<int32_t>(ns);
    std::vector<uint64_t> hsig;
    uint64_t *table = nullptr;
    for (;;) {
        table = a.get_n<uint64_t>((int64_t)H + 1);
        HIP_CHECK(hipMemsetAsync(table, 0xff, 8 * H, s));
        fill_i32(reinterpret_cast<int32_t *>(table + H), 0, 2, s);
        hipLaunchKernelGGL(k_sig_insert, grid1(ns), 256, 0, s, (const uint64_t *)sig, ns, table, H - 1, at,
                           reinterpret_cast<int32_t *>(table + H));
        const uint64_t cap = H / 2;
        unsigned long long *kc = a.get_n<unsigned long long>((int64_t)cap + 2);
        fill_i32(reinterpret_cast<int32_t *>(kc), 0, 2, s);
        hipLaunchKernelGGL(k_key_compact, std::min(grid1((int64_t)H), 1024), 256, 0, s, (const uint64_t *)table, H, cap,
                           kc);
        const int64_t kbytes = 8 * ((int64_t)cap + 2);
        std::vector<unsigned long long> hbuf(cap + 2);
        if (kbytes <= Mailbox::kFetchBytes) {
            std::memcpy(hbuf.data(), mb.fetch(kc, kbytes, s), kbytes);
        } else {
            HIP_CHECK(hipMemcpyAsync(hbuf.data(), kc, kbytes, hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
        }
        a.put(kc);
        int32_t hf[2];
        std::memcpy(hf, &hbuf[1], 8);
        const int64_t used = (int64_t)hbuf[0];
        if (!hf[1] && 2 * used <= (int64_t)H) {
            hsig.assign(hbuf.begin() + 2, hbuf.begin() + 2 + used);
            break;
        }
        a.put(table);
        H *= 4;
    }
    a.put(err);
    std::sort(hsig.begin(), hsig.end());
    const int64_t nsig = (int64_t)hsig.size();
    st.nsig = nsig;
    if (!keep && ns < (int64_t)kSlotsPerSig * nsig) {
        // slots with this many key sequences fill their tiles poorly: the pairs stay in the
        // target tiles (the caller rebuilds the dense cells)
        a.put(table); a.put(at); a.put(sig);
        st.release(a);
        st.abandoned = true;
        lg("  slots: given up (diverse signatures)");
        return;
    }
    uint64_t *dsig = a.get_n<uint64_t>(nsig);
    mb.upload(dsig, hsig.data(), 8 * nsig, s);
    int32_t *tslot = a.get_n<int32_t>((int64_t)H);
    hipLaunchKernelGGL(k_slot_ids, grid1((int64_t)H), 256, 0, s, (const uint64_t *)table, H, (const uint64_t *)dsig,
                       nsig, tslot);
    int32_t *sig_id = a.get_n<int32_t>(ns);
    hipLaunchKernelGGL(k_sig_ids, grid1(ns), 256, 0, s, (const int32_t *)at, (const int32_t *)tslot, ns, sig_id);
    a.put(tslot); a.put(table); a.put(dsig); a.put(at); a.put(sig);
    lg("  slots: signatures");

    // tile order: (region, signature, target); tiles of 64 slots inside each (region, signature)
    int rl = kSlotRegionLevel;
    if (const char *ev = getenv("FMM_M2L_REGION_LEVEL")) rl = std::max(0, std::min(6, atoi(ev)));
    const int sbits = bits_for(nsig);
    if (3 * rl + sbits > 64) rl = std::max(0, (64 - sbits) / 3);
    uint64_t *tk = a.get_n<uint64_t>(ns);
    st.sorted = a.get_n<int32_t>(ns);
    hipLaunchKernelGGL(k_slot_sort_keys, grid1(ns), 256, 0, s, (const int32_t *)st.slot_tgt, (const int32_t *)sig_id, ns,
                       C, rl, sbits, tk, st.sorted);
    radix_sort_u64(tk, st.sorted, ns, 3 * rl + sbits, a, s);
    st.gflag = a.get_n<int32_t>(ns);
    st.gid = a.get_n<int32_t>(ns);
    hipLaunchKernelGGL(k_group_flags, grid1(ns), 256, 0, s, (const uint64_t *)tk, ns, st.gflag);
    a.put(tk);
    const int64_t ngroups = exclusive_scan_i32(st.gflag, st.gid, ns, a, s);
    st.gstart = a.get_n<int32_t>(ngroups);
    hipLaunchKernelGGL(k_group_starts, grid1(ns), 256, 0, s, (const int32_t *)st.gflag, (const int32_t *)st.gid, ns,
                       st.gstart);
    {   // key sequence of every signature, from a representative slot
        int32_t *rep = a.get_n<int32_t>(nsig);
        hipLaunchKernelGGL(k_group_rep, grid1(ns), 256, 0, s, (const int32_t *)st.gflag, (const int32_t *)st.sorted,
                           (const int32_t *)sig_id, ns, rep);
        st.sig_keys = a.get_n<int32_t>(8 * nsig);
        st.sig_n = a.get_n<int32_t>(nsig);
        hipLaunchKernelGGL(k_sig_keys, grid1(nsig), 256, 0, s, (const int32_t *)rep, nsig,
                           (const int32_t *)st.slot_first, (const int32_t *)st.slot_mb, key_id, st.sig_keys, st.sig_n);
        a.put(rep);
    }
    st.tflag = a.get_n<int32_t>(ns);
    st.tid = a.get_n<int32_t>(ns);
    hipLaunchKernelGGL(k_tile_flags, grid1(ns), 256, 0, s, (const int32_t *)st.gflag, (const int32_t *)st.gid,
                       (const int32_t *)st.gstart, ns, st.tflag);
    const int64_t nt = exclusive_scan_i32(st.tflag, st.tid, ns, a, s);
    st.ntiles = nt;
    st.tile_sig = a.get_n<int32_t>(nt);
    st.tile_ne = a.get_n<int32_t>(nt);
    st.tile_eoff = a.get_n<int32_t>(nt);
    hipLaunchKernelGGL(k_tile_sig, grid1(ns), 256, 0, s, (const int32_t *)st.tflag, (const int32_t *)st.tid,
                       (const int32_t *)st.sorted, (const int32_t *)sig_id, (const int32_t *)st.sig_n, ns, st.tile_sig,
                       st.tile_ne);
    a.put(sig_id);
    st.ne = exclusive_scan_i32(st.tile_ne, st.tile_eoff, nt, a, s);
    lg("  slots: tiles");
    if (st.ne + 1 >= (int64_t(1) << 31) / kTileN) fail(FMM_EUNSUPPORTED, "too many M2L slot entries");

    // the fixed-order sum: runs of slots of one target (slots are numbered in target order)
    P->slot_pos = a.get_n<int64_t>(ns);
    int32_t *rflag = a.get_n<int32_t>(ns), *rid = a.get_n<int32_t>(ns);
    hipLaunchKernelGGL(k_run_flags, grid1(ns), 256, 0, s, (const int32_t *)st.slot_tgt, ns, rflag);
    const int64_t nr = exclusive_scan_i32(rflag, rid, ns, a, s);
    P->nruns = nr;
    P->run_first = a.get_n<int32_t>(nr + 1);
    P->run_tgt = a.get_n<int32_t>(nr);
    hipLaunchKernelGGL(k_run_info, grid1(ns), 256, 0, s, (const int32_t *)rflag, (const int32_t *)rid,
                       (const int32_t *)st.slot_tgt, ns, P->run_first, P->run_tgt);
    {
        const int32_t end = (int32_t)ns;
        mb.upload(P->run_first + nr, &end, 4, s);
    }
    a.put(rflag); a.put(rid);
    lg("  slots: runs");
    if (lg.on)
        fprintf(stderr, "[fmm plan]   pool %lld pairs, %lld slots, %lld signatures, %lld groups, %lld tiles, %lld entries\n",
                (long long)npool, (long long)ns, (long long)nsig, (long long)ngroups, (long long)nt, (long long)st.ne);
}

// Host-side range checks of the M2L grouping (FMM_VALIDATE_PLAN set): every index an
// evaluation kernel will follow is checked before any evaluation runs.
template <class T> static std::vector<T> dl(const T *dev, int64_t n, hipStream_t s) {
    std::vector<T> h((size_t)std::max<int64_t>(n, 0));
    if (n > 0) HIP_CHECK(hipMemcpyAsync(h.data(), dev, sizeof(T) * n, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return h;
}
static void validate_m2l(fmm_plan_s *P, hipStream_t s) {
    if (P->nm2l == 0) return;
    const int64_t nc = P->ncells, ne = P->nentries, nw = P->nwork, np = P->npartial, nt = P->ntiles;
    char msg[256];
    auto bad = [&](const char *what, int64_t i, int64_t v) {
        snprintf(msg, sizeof msg, "plan validation: %s at %lld = %lld (nc %lld ne %lld nwork %lld npartial %lld "
                 "ntiles %lld nkeys %lld nslots %lld nruns %lld)", what, (long long)i, (long long)v, (long long)nc,
                 (long long)ne, (long long)nw, (long long)np, (long long)nt, (long long)P->nkeys,
                 (long long)P->nslots, (long long)P->nruns);
        fail(FMM_EDEVICE, msg);
    };
    auto w = dl(P->work, nw, s);
    for (int64_t i = 0; i < nw; ++i) {
        if (w[i].y < 0 || w[i].z > ne || w[i].y > w[i].z) bad("work entry range", i, w[i].y);
        if (w[i].w < 0 || w[i].w > np) bad("work partial", i, w[i].w);
        if (w[i].w == 0 && (w[i].x < 0 || w[i].x >= nt)) bad("work tile", i, w[i].x);
    }
    auto ek = dl(P->entry_key, ne, s);
    for (int64_t e = 0; e < ne; ++e)
        if (ek[e] < 0 || ek[e] >= P->nkeys) bad("entry key", e, ek[e]);
    auto es = dl(P->entry_src, ne * kTileN, s);
    auto em = dl(P->entry_mask, ne, s);
    int64_t nsrc = 0;
    for (int64_t e = 0; e < ne; ++e) {
        int m = 0;
        for (int l = 0; l < kTileN; ++l) {
            const int v = es[e * kTileN + l];
            if (v < -1 || v >= nc) bad("entry source", e * kTileN + l, v);
            if (v >= 0) m |= 1 << (l / 16);
            nsrc += v >= 0;
        }
        if (m != em[e]) bad("entry mask", e, em[e]);
    }
    if (nsrc != P->nm2l) bad("entry columns with a source (every M2L pair once)", 0, nsrc);
    auto tt = dl(P->tile_targets, nt * kTileN, s);
    for (int64_t i = 0; i < nt * kTileN; ++i)
        if (tt[i] < -1 || tt[i] >= nc) bad("tile target", i, tt[i]);
    auto tw = dl(P->tile_work, nt + 1, s);
    for (int64_t t = 0; t < nt; ++t)
        if (tw[t] > tw[t + 1]) bad("tile work order", t, tw[t]);
    if (P->nslots > 0) {
        auto sp = dl(P->slot_pos, P->nslots, s);
        for (int64_t q = 0; q < P->nslots; ++q)
            if (sp[q] < 0 || sp[q] >= np * kTileN) bad("slot position", q, sp[q]);
        auto rf = dl(P->run_first, P->nruns + 1, s);
        auto rt = dl(P->run_tgt, P->nruns, s);
        if (rf[0] != 0 || rf[P->nruns] != P->nslots) bad("run bounds", 0, rf[P->nruns]);
        for (int64_t r = 0; r < P->nruns; ++r) {
            if (rf[r] >= rf[r + 1]) bad("run order", r, rf[r]);
            if (rt[r] < 0 || rt[r] >= nc) bad("run target", r, rt[r]);
        }
    }
    auto kp = dl(P->key_f32, P->nkeys, s);
    for (int64_t k = 0; k < P->nkeys; ++k)
        if (!kp[k]) bad("operator pointer", k, 0);
    fprintf(stderr, "[fmm validate] ok: nc %lld entries %lld work %lld partial %lld tiles %lld pool %lld slots %lld "
            "slot tiles %lld runs %lld\n", (long long)nc, (long long)ne, (long long)nw, (long long)np, (long long)nt,
            (long long)P->npool, (long long)P->nslots, (long long)P->nslot_tiles, (long long)P->nruns);
}

void build_plan(fmm_plan_s *P, const float *points, hipStream_t s) {
    StageLog lg;
    lg.s = s;
    Alloc &a = P->mem;
    const int64_t n = P->n;
    // small results come back through a mailbox; the stream is drained before it is
    // handed back (its upload arena may still be read by queued copies after a failure)
    MailboxLease lease;
    Mailbox &mb = *lease.m;
    struct Drain {
        Alloc &a;
        hipStream_t s;
        ~Drain() {
            (void)hipStreamSynchronize(s);
            a.mb = nullptr;
        }
    } drain{a, s};
    a.mb = &mb;
    // counted on the device, read once at the end: same-level M2L pairs, P2P interactions,
    // near-field runs, near-field work items, partial blocks, total run length
    unsigned long long *counts = a.get_n<unsigned long long>(6);
    fill_i32(reinterpret_cast<int32_t *>(counts), 0, 12, s);

    // ---- a1: root cube and keys
    int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    float *bpart = a.get_n<float>(8 * nb);
    hipLaunchKernelGGL(k_bbox_partial, nb, 256, 0, s, points, n, bpart);
    float hb[8];
    {
        const uint64_t t = mb.next_ticket();
        hipLaunchKernelGGL(k_bbox_final, 1, 256, 0, s, (const float *)bpart, nb, mb.data_dev<float>(), mb.flag_dev(), t);
        mb.wait(t, s);
        std::memcpy(hb, mb.data_host<float>(), sizeof(float) * 7);
    }
    a.put(bpart);
    if (hb[6] != 0.f) fail(FMM_ENONFINITE, "a coordinate is NaN or infinite");
    root_cube(hb, hb + 3, P->k, P->x0);

    uint64_t *keys = a.get_n<uint64_t>(n);
    int32_t *perm = a.get_n<int32_t>(n);
    hipLaunchKernelGGL(k_keys, grid1(n), 256, 0, s, points, n, P->x0[0], P->x0[1], P->x0[2],
                       std::ldexp(1.0, kMaxLevel - P->k), keys, perm);
    lg("bbox+keys");
    // ---- a2: sort (stable: equal keys keep input order) and permute
    radix_sort_u64(keys, perm, n, 3 * kMaxLevel, a, s);
    P->keys = keys;
    P->perm = perm;
    P->iperm = a.get_n<int32_t>(n);
    hipLaunchKernelGGL(k_invert_perm, grid1(n), 256, 0, s, (const int32_t *)perm, n, P->iperm);
    P->bodies = a.get_n<float4>(n);
    hipLaunchKernelGGL(k_gather_bodies, grid1(n), 256, 0, s, points, (const int32_t *)perm, n, P->bodies);

    lg("sort+permute");
    // ---- a3: octree, level by level, written straight into the global cell arrays
    // (level l occupies [level_off[l], level_off[l+1]); arrays grow by doubling)
    int64_t cap = std::max<int64_t>(4096, 8 * n / std::max(1, P->ncrit) + 64);
    uint64_t *c_prefix = a.get_n<uint64_t>(cap);
    int32_t **c32[9] = {&P->c_ix, &P->c_iy, &P->c_iz, &P->c_start, &P->c_count, &P->c_parent, &P->c_nchild,
                        &P->c_child0, &P->c_level};
    for (int q = 0; q < 9; ++q) *c32[q] = a.get_n<int32_t>(cap);
    auto ensure = [&](int64_t used, int64_t need) {
        if (need <= cap) return;
        int64_t c2 = cap;
        grow(a, c_prefix, c2, used, need, s);
        for (int q = 0; q < 9; ++q) {
            c2 = cap;
            grow(a, *c32[q], c2, used, need, s);
        }
        cap = c2;
    };
    hipLaunchKernelGGL(k_init_root, 1, 64, 0, s, (int32_t)n, c_prefix, P->c_ix, P->c_iy, P->c_iz, P->c_start,
                       P->c_count, P->c_parent, P->c_level);
    std::vector<int64_t> level_off{0, 1};
    for (int l = 0;; ++l) {
        const int64_t o0 = level_off[l], o1 = level_off[l + 1], m = o1 - o0;
        int32_t *cs8 = a.get_n<int32_t>(8 * m), *cc8 = a.get_n<int32_t>(8 * m), *off = a.get_n<int32_t>(m);
        hipLaunchKernelGGL(k_split, grid1(8 * m), 256, 0, s, m, (const int32_t *)P->c_start + o0,
                           (const int32_t *)P->c_count + o0, (const uint64_t *)c_prefix + o0, l, P->ncrit,
                           (const uint64_t *)keys, P->c_nchild + o0, cs8, cc8);
        const int64_t nnext = exclusive_scan_i32(P->c_nchild + o0, off, m, a, s);
        ensure(o1, o1 + nnext);
        hipLaunchKernelGGL(k_write_children, grid1(m), 256, 0, s, m, o0, o1, (const int32_t *)P->c_nchild + o0,
                           (const int32_t *)off, (const int32_t *)cs8, (const int32_t *)cc8,
                           (const uint64_t *)c_prefix + o0, (const int32_t *)P->c_ix + o0,
                           (const int32_t *)P->c_iy + o0, (const int32_t *)P->c_iz + o0, P->c_child0 + o0,
                           c_prefix + o1, P->c_ix + o1, P->c_iy + o1, P->c_iz + o1, P->c_start + o1, P->c_count + o1,
                           P->c_parent + o1, P->c_level + o1, l + 1);
        a.put(cs8); a.put(cc8); a.put(off);
        if (nnext == 0) break;
        level_off.push_back(o1 + nnext);
    }
    P->max_level = (int)level_off.size() - 2;
    P->level_off = level_off;
    const int64_t nc = level_off.back();
    P->ncells = nc;
    P->c_prefix_dev = c_prefix;

    lg("octree");
    // leaves
    {
        int32_t *flag = a.get_n<int32_t>(nc), *ex = a.get_n<int32_t>(nc);
        hipLaunchKernelGGL(k_leaf_flags, grid1(nc), 256, 0, s, (const int32_t *)P->c_nchild, nc, flag);
        P->nleaves = exclusive_scan_i32(flag, ex, nc, a, s);
        P->leaves = a.get_n<int32_t>(P->nleaves);
        P->leaf_id = a.get_n<int32_t>(nc);
        hipLaunchKernelGGL(k_leaf_compact, grid1(nc), 256, 0, s, (const int32_t *)flag, (const int32_t *)ex, nc,
                           P->leaves, P->leaf_id);
        a.put(flag); a.put(ex);
        P->body_leaf = a.get_n<int32_t>(n);
        hipLaunchKernelGGL(k_body_leaf, (int)std::min<int64_t>(P->nleaves, 65536), 64, 0, s,
                           (const int32_t *)P->leaves, P->nleaves, (const int32_t *)P->c_start,
                           (const int32_t *)P->c_count, P->body_leaf);
    }

    lg("leaves");
    CellView C{P->c_level, P->c_ix, P->c_iy, P->c_iz, P->c_child0, P->c_nchild, P->c_prefix_dev, P->lists};
    uint8_t *ckind = nullptr;
    if (P->ntgt > 0) {
        // separate target set: which cells hold sources and which targets, so that the
        // traversal keeps only the pairs that carry a field to a target or an adjoint
        // weight to a source
        int32_t *flag = a.get_n<int32_t>(n), *pre = a.get_n<int32_t>(n + 1);
        hipLaunchKernelGGL(k_src_flags, grid1(n), 256, 0, s, (const int32_t *)P->perm, n, P->nsrc, flag);
        exclusive_scan_i32(flag, pre, n, a, s);
        {
            const int32_t tot = (int32_t)P->nsrc;
            mb.upload(pre + n, &tot, 4, s);
        }
        ckind = a.get_n<uint8_t>(nc);
        hipLaunchKernelGGL(k_cell_kind, grid1(nc), 256, 0, s, (const int32_t *)P->c_start, (const int32_t *)P->c_count,
                           nc, (const int32_t *)pre, ckind);
        a.put(flag); a.put(pre);
        C.kind = ckind;
    }

    // ---- M2M and L2L as grouped GEMMs: per-level tiles of parents (M2M) and of
    // same-octant children (L2L)
    {
        int32_t *flag = a.get_n<int32_t>(nc);
        int32_t *ct = a.get_n<int32_t>(nc), *cl = a.get_n<int32_t>(nc);
        int64_t ntg = 0;
        hipLaunchKernelGGL(k_flag_internal, grid1(nc), 256, 0, s, (const int32_t *)P->c_nchild, nc, flag);
        P->m2m.ntiles = tile_cells(C, nc, flag, false, false, a, s, P->m2m.tile_targets, ct, cl, P->m2m.bucket_tile, ntg);
        if (P->m2m.ntiles > 0) {
            P->m2m.entry_src = a.get_n<int32_t>(P->m2m.ntiles * 8 * kTileN);
            fill_i32(P->m2m.entry_src, -1, P->m2m.ntiles * 8 * kTileN, s);
            P->m2m.entry_key = a.get_n<int32_t>(P->m2m.ntiles * 8);
            P->m2m.work = a.get_n<int4>(P->m2m.ntiles);
            hipLaunchKernelGGL(k_m2m_entries, grid1(nc), 256, 0, s, nc, C, (const int32_t *)ct, (const int32_t *)cl,
                               P->m2m.entry_src);
            hipLaunchKernelGGL(k_work_uniform, grid1(P->m2m.ntiles), 256, 0, s, P->m2m.ntiles, 8, P->m2m.entry_key,
                               P->m2m.work);
        }
        hipLaunchKernelGGL(k_flag_nonroot, grid1(nc), 256, 0, s, (const int32_t *)P->c_level, nc, flag);
        P->l2l.ntiles = tile_cells(C, nc, flag, true, false, a, s, P->l2l.tile_targets, ct, cl, P->l2l.bucket_tile, ntg);
        if (P->l2l.ntiles > 0) {
            P->l2l.entry_src = a.get_n<int32_t>(P->l2l.ntiles * kTileN);
            fill_i32(P->l2l.entry_src, -1, P->l2l.ntiles * kTileN, s);
            P->l2l.entry_key = a.get_n<int32_t>(P->l2l.ntiles);
            P->l2l.work = a.get_n<int4>(P->l2l.ntiles);
            hipLaunchKernelGGL(k_l2l_entries, grid1(nc), 256, 0, s, nc, C, (const int32_t *)P->c_parent,
                               (const int32_t *)ct, (const int32_t *)cl, P->l2l.entry_key, P->l2l.entry_src);
            hipLaunchKernelGGL(k_work_uniform, grid1(P->l2l.ntiles), 256, 0, s, P->l2l.ntiles, 1, (int32_t *)nullptr,
                               P->l2l.work);
        }
        a.put(flag); a.put(ct); a.put(cl);
    }

    lg("m2m/l2l tiles");
    // ---- a4: dual traversal, one fused step per level of the pair tree
    const double theta2 = (double)P->theta * (double)P->theta;
    unsigned long long *cnt = a.get_n<unsigned long long>(4);
    fill_i32(reinterpret_cast<int32_t *>(cnt), 0, 8, s);
    int2 *m2l = nullptr, *p2p = nullptr;
    int32_t *m2l_slot = nullptr;
    int4 *recs = nullptr;
    int64_t m2l_cap = 0, slot_cap = 0, rec_cap = 0, p2p_cap = 0, nm2l = 0, np2p = 0, nrec = 0;
    // operator-key table filled by the traversal (its last word holds the two flags),
    // M2L targets marked by it
    const uint64_t H0 = uint64_t(1) << 16;
    uint64_t *ktable = nullptr;
    int32_t *is_t = nullptr;
    if (nc == 1) {               // the root is a leaf: one P2P pair
        grow(a, p2p, p2p_cap, 0, 1, s);
        fill_i32(reinterpret_cast<int32_t *>(p2p), 0, 2, s);
        np2p = 1;
    } else {
        // first guess of the list sizes (a uniform cloud at theta = 0.4 has ~350-450 M2L
        // pairs per cell in ~50-90 slots and ~75 P2P pairs per leaf); the M2L list starts
        // large enough for the worst-case reserve of the largest step of such a cloud (64
        // per split pair, ~14.5M split pairs at 2^24 points), so that it is not grown (and
        // copied) during the traversal; a step that overflows is repeated
        grow(a, m2l, m2l_cap, 0, 1024 * nc, s);
        grow(a, m2l_slot, slot_cap, 0, m2l_cap, s);
        grow(a, recs, rec_cap, 0, 128 * nc, s);
        grow(a, p2p, p2p_cap, 0, 96 * P->nleaves + 64, s);
        ktable = a.get_n<uint64_t>((int64_t)H0 + 1);
        HIP_CHECK(hipMemsetAsync(ktable, 0xff, 8 * H0, s));
        fill_i32(reinterpret_cast<int32_t *>(ktable + H0), 0, 2, s);
        is_t = a.get_n<int32_t>(nc);
        fill_i32(is_t, 0, nc, s);
        int2 *front = a.get_n<int2>(1);
        fill_i32(reinterpret_cast<int32_t *>(front), 0, 2, s);
        int64_t nf = 1;
        while (nf > 0) {
            // steady state of a uniform tree: ~8 split pairs, ~56 M2L pairs in ~12 slots and
            // ~8 P2P pairs per split pair
            int64_t cap_n = std::max<int64_t>(1024, std::min<int64_t>(64 * nf, 10 * nf));
            grow(a, m2l, m2l_cap, nm2l, nm2l + 64 * nf, s);
            grow(a, m2l_slot, slot_cap, nm2l, m2l_cap, s);
            grow(a, recs, rec_cap, nrec, nrec + 8 * nf, s);   // a record per target child at most
            grow(a, p2p, p2p_cap, np2p, np2p + 12 * nf, s);
            int2 *next = a.get_n<int2>(cap_n);
            uint64_t h4[4];
            for (int attempt = 0;; ++attempt) {
                const int64_t per_block = 4 * kTravPerWave;
                const int64_t tb = (nf + per_block - 1) / per_block;
                if (tb >= (int64_t(1) << 31)) fail(FMM_EUNSUPPORTED, "traversal frontier too large");
                const uint64_t t = mb.next_ticket();
                const TravOut to{m2l, m2l_slot, std::min(m2l_cap, slot_cap), recs, rec_cap, p2p, p2p_cap, next, cap_n,
                                 ktable, H0 - 1, reinterpret_cast<int32_t *>(ktable + H0), is_t};
                hipLaunchKernelGGL(k_trav_step, (int)tb, 256, 0, s, C, (const int2 *)front, nf, theta2, cnt, to);
                hipLaunchKernelGGL(k_trav_post, 1, 64, 0, s, cnt, mb.data_dev<unsigned long long>(), mb.flag_dev(), t);
                mb.wait(t, s);
                std::memcpy(h4, mb.data_host<uint64_t>(), sizeof(h4));
                bool ok = (int64_t)h4[0] <= std::min(m2l_cap, slot_cap) && (int64_t)h4[1] <= p2p_cap &&
                          (int64_t)h4[2] <= cap_n && (int64_t)h4[3] <= rec_cap;
                if (ok) break;
                if (attempt > 0) fail(FMM_EDEVICE, "traversal step overflowed twice");
                hipLaunchKernelGGL(k_set_counters, 1, 64, 0, s, cnt, nm2l, np2p, nrec);
                grow(a, m2l, m2l_cap, nm2l, (int64_t)h4[0], s);
                grow(a, m2l_slot, slot_cap, nm2l, m2l_cap, s);
                grow(a, recs, rec_cap, nrec, (int64_t)h4[3], s);
                grow(a, p2p, p2p_cap, np2p, (int64_t)h4[1], s);
                if ((int64_t)h4[2] > cap_n) {
                    a.put(next);
                    cap_n = (int64_t)h4[2];
                    next = a.get_n<int2>(cap_n);
                }
            }
            nm2l = (int64_t)h4[0];
            np2p = (int64_t)h4[1];
            nrec = (int64_t)h4[3];
            a.put(front);
            front = next;
            nf = (int64_t)h4[2];
        }
        a.put(front);
    }
    a.put(cnt);
    if (ckind) a.put(ckind);
    P->nm2l = nm2l;
    P->np2p = np2p;
    P->m2l_pairs = m2l;

    // ---- P2P lists, on the side stream while the host builds the M2L grouping: no host
    // waits (the run count stays on the device; the run array is sized for one run per
    // pair).  Temporaries come from an allocator bound to the side stream; everything it
    // still holds joins the plan's workspace when the build ends.
    struct SideAlloc {
        Alloc &main;
        Alloc as;
        ~SideAlloc() {
            main.live.insert(main.live.end(), as.live.begin(), as.live.end());
            main.bytes += as.bytes;
        }
    } side{a, Alloc{}};
    int32_t *p2p_pieces = nullptr, *p2p_part_len = nullptr, *p2p_item_off = nullptr, *p2p_part_off = nullptr;
    {
        Alloc &as = side.as;
        as.alloc = a.alloc;
        as.release = a.release;
        as.ctx = a.ctx;
        as.stream = P->side;
        hipStream_t ss = P->side;
        HIP_CHECK(hipEventRecord(P->ev_fork, s));
        HIP_CHECK(hipStreamWaitEvent(ss, P->ev_fork, 0));
        uint64_t *comp = as.get_n<uint64_t>(np2p);
        int32_t *dummy = as.get_n<int32_t>(np2p);
        const int lbits = bits_for(P->nleaves);
        hipLaunchKernelGGL(k_p2p_composite, grid1(np2p), 256, 0, ss, (const int2 *)p2p, np2p,
                           (const int32_t *)P->leaf_id, lbits, comp, dummy);
        radix_sort_u64(comp, dummy, np2p, 2 * lbits, as, ss);
        P->p2p_pairs = as.get_n<int2>(np2p);
        int32_t *pair_off = as.get_n<int32_t>(P->nleaves);
        hipLaunchKernelGGL(k_p2p_csr, std::min(grid1(np2p), 1024), 256, 0, ss, (const uint64_t *)comp,
                           (const int32_t *)dummy, np2p, lbits, (const int32_t *)P->leaves, P->p2p_pairs, pair_off,
                           (const int32_t *)P->c_count, &counts[1]);
        // runs: open flags in `dummy` (free after the CSR pass), run ids in `comp`'s storage
        int32_t *open = dummy, *run_id = reinterpret_cast<int32_t *>(comp);
        hipLaunchKernelGGL(k_p2p_run_flags, grid1(np2p), 256, 0, ss, (const int2 *)P->p2p_pairs, np2p,
                           (const int32_t *)P->c_start, (const int32_t *)P->c_count, open);
        int64_t *nseg_dev = reinterpret_cast<int64_t *>(&counts[2]);
        exclusive_scan_i32_to(open, run_id, np2p, nseg_dev, as, ss);
        P->seg_off = as.get_n<int32_t>(P->nleaves + 1);
        P->segs = as.get_n<int2>(np2p);
        hipLaunchKernelGGL(k_p2p_run_write, grid1(np2p), 256, 0, ss, (const int2 *)P->p2p_pairs, np2p,
                           (const int32_t *)P->c_start, (const int32_t *)P->c_count, (const int32_t *)open,
                           (const int32_t *)run_id, P->segs);
        hipLaunchKernelGGL(k_p2p_run_len, grid1(np2p), 256, 0, ss, P->segs, (const int64_t *)nseg_dev);
        hipLaunchKernelGGL(k_p2p_seg_off, grid1(P->nleaves + 1), 256, 0, ss, (int64_t)P->nleaves,
                           (const int32_t *)pair_off, (const int32_t *)run_id, (const int64_t *)nseg_dev, P->seg_off);
        as.put(comp); as.put(dummy); as.put(pair_off);
        // work items of the near field (heavy leaves split into pieces): counts of items and
        // partial blocks go to counts[3], counts[4]; the items are written after the join
        int64_t *lens = as.get_n<int64_t>(np2p + 1);
        hipLaunchKernelGGL(k_p2p_run_len64, grid1(np2p + 1), 256, 0, ss, (const int2 *)P->segs,
                           (const int64_t *)nseg_dev, np2p + 1, lens);
        P->run_pre = as.get_n<int64_t>(np2p + 1);
        exclusive_scan_i64_to(lens, P->run_pre, np2p + 1, reinterpret_cast<int64_t *>(&counts[5]), as, ss);
        as.put(lens);
        p2p_pieces = as.get_n<int32_t>(P->nleaves);
        p2p_part_len = as.get_n<int32_t>(P->nleaves);
        p2p_item_off = as.get_n<int32_t>(P->nleaves);
        p2p_part_off = as.get_n<int32_t>(P->nleaves);
        hipLaunchKernelGGL(k_p2p_split, grid1(P->nleaves), 256, 0, ss, (int64_t)P->nleaves, (const int32_t *)P->leaves,
                           (const int32_t *)P->c_count, (const int32_t *)P->seg_off, (const int64_t *)P->run_pre,
                           p2p_pieces, p2p_part_len);
        exclusive_scan_i32_to(p2p_pieces, p2p_item_off, P->nleaves, reinterpret_cast<int64_t *>(&counts[3]), as, ss);
        exclusive_scan_i32_to(p2p_part_len, p2p_part_off, P->nleaves, reinterpret_cast<int64_t *>(&counts[4]), as, ss);
    }

    lg("traversal");
    // ---- M2L keys, operators, tiles, entries
    if (nm2l > 0) {
        if (nm2l >= (int64_t(1) << 31)) fail(FMM_EUNSUPPORTED, "more than 2^31 M2L pairs");
        // target tiles (targets marked by the traversal)
        int32_t *cell_tile = a.get_n<int32_t>(nc), *cell_lane = a.get_n<int32_t>(nc);
        std::vector<int32_t> btile;
        int64_t ntiles = tile_cells(C, nc, is_t, true, true, a, s, P->tile_targets, cell_tile, cell_lane, btile, P->ntargets);
        P->ntiles = ntiles;
        a.put(is_t);
        lg("m2l target tiles");

        // distinct operator keys through a device hash table; every pair keeps its slot
        // (the table's last word holds the two flags: key out of range, table full).  The
        // traversal has filled the first table; a fuller one is rebuilt larger from the pairs.
        uint64_t H = H0;
        int32_t *pkid = m2l_slot;
        uint64_t *table = ktable;
        std::vector<uint64_t> hkeys;
        for (;;) {
            if (!table) {
                table = a.get_n<uint64_t>((int64_t)H + 1);
                HIP_CHECK(hipMemsetAsync(table, 0xff, 8 * H, s));
                fill_i32(reinterpret_cast<int32_t *>(table + H), 0, 2, s);
                hipLaunchKernelGGL(k_key_insert, grid1(nm2l), 256, 0, s, (const int2 *)m2l, nm2l, C, table, H - 1,
                                   pkid, reinterpret_cast<int32_t *>(table + H));
            }
            // the distinct keys, compacted on the device (a table holding more than H / 2
            // of them is rebuilt larger, so cap = H / 2 keeps every key of an accepted one)
            const uint64_t cap = H / 2;
            unsigned long long *kc = a.get_n<unsigned long long>((int64_t)cap + 2);
            fill_i32(reinterpret_cast<int32_t *>(kc), 0, 2, s);
            hipLaunchKernelGGL(k_key_compact, std::min(grid1((int64_t)H), 1024), 256, 0, s, (const uint64_t *)table, H,
                               cap, kc);
            const int64_t kbytes = 8 * ((int64_t)cap + 2);
            std::vector<unsigned long long> hbuf;
            const unsigned long long *hk;
            if (kbytes <= Mailbox::kFetchBytes) {
                hk = static_cast<const unsigned long long *>(mb.fetch(kc, kbytes, s));
            } else {
                hbuf.resize(cap + 2);
                HIP_CHECK(hipMemcpyAsync(hbuf.data(), kc, kbytes, hipMemcpyDeviceToHost, s));
                HIP_CHECK(hipStreamSynchronize(s));
                hk = hbuf.data();
            }
            int32_t hf[2];
            std::memcpy(hf, &hk[1], 8);
            if (hf[0]) fail(FMM_EUNSUPPORTED, "an M2L offset exceeds the key range");
            const int64_t used = (int64_t)hk[0];
            if (!hf[1] && 2 * used <= (int64_t)H) {
                hkeys.assign(hk + 2, hk + 2 + used);
                a.put(kc);
                break;
            }
            a.put(kc);
            a.put(table);
            table = nullptr;
            H *= 4;
        }
        std::sort(hkeys.begin(), hkeys.end());
        const int64_t nkeys = (int64_t)hkeys.size();
        P->nkeys = nkeys;
        std::vector<int32_t> hsame(nkeys);
        P->nkeys_same = 0;
        for (int64_t k2 = 0; k2 < nkeys; ++k2) {
            hsame[k2] = (int(hkeys[k2] >> 57) - 32) == 0;
            P->nkeys_same += hsame[k2];
        }
        std::vector<uint64_t> p32, p16;
        m2l_operator_ptrs(P->p, hkeys, p32, p16, P->prec == FMM_PREC_MIXED);
        uint64_t *d32 = a.get_n<uint64_t>(nkeys);
        mb.upload(d32, p32.data(), 8 * nkeys, s);
        P->key_f32 = d32;
        if (P->prec == FMM_PREC_MIXED) {
            uint64_t *d16 = a.get_n<uint64_t>(nkeys);
            mb.upload(d16, p16.data(), 8 * nkeys, s);
            P->key_f16 = d16;
        }
        std::vector<float> key_kept;   // per key: fraction of the dense operator's flops applied
        std::vector<int32_t> svd_rank;
        if (P->m2l_tol > 0) {
            std::vector<uint32_t> rows;
            m2l_block_rows(P->p, hkeys, P->m2l_tol, rows, key_kept);
            P->key_rows = a.get_n<uint32_t>((int64_t)rows.size());
            mb.upload(P->key_rows, rows.data(), 4 * rows.size(), s);
        } else if (P->svd_tol > 0) {
            // SVD-compressed operators: two products of rank r cost 4 r NC flop per pair
            std::vector<uint64_t> sp;
            std::vector<int32_t> rpad;
            m2l_svd_ptrs(P->p, hkeys, P->svd_tol, sp, rpad, svd_rank);
            uint64_t *dsp = a.get_n<uint64_t>(2 * nkeys);
            mb.upload(dsp, sp.data(), 8 * sp.size(), s);
            P->key_svd = dsp;
            P->key_rank = a.get_n<int32_t>(nkeys);
            mb.upload(P->key_rank, rpad.data(), 4 * nkeys, s);
            key_kept.resize(nkeys);
            for (int64_t k2 = 0; k2 < nkeys; ++k2) key_kept[k2] = (float)(2.0 * svd_rank[k2] / ncoef(P->p));
        }
        uint64_t *dkeys = a.get_n<uint64_t>(nkeys);
        mb.upload(dkeys, hkeys.data(), 8 * nkeys, s);
        int32_t *slot_id = a.get_n<int32_t>((int64_t)H);
        hipLaunchKernelGGL(k_slot_ids, grid1((int64_t)H), 256, 0, s, (const uint64_t *)table, H, (const uint64_t *)dkeys,
                           nkeys, slot_id);
        int32_t *dsame = a.get_n<int32_t>(nkeys);
        mb.upload(dsame, hsame.data(), 4 * nkeys, s);
        lg("m2l keys+operators");

        // (tile, key) cells: the target lanes of each, through a 64-bit mask per cell.  Cells
        // whose sources fill their 16-column blocks well become entries of their target tile
        // (tile-major, key-ascending); the pairs of the others go to the slot pool.
        const int64_t ntk = ntiles * nkeys;
        if (ntk >= (int64_t(1) << 31)) fail(FMM_EUNSUPPORTED, "M2L tile x key table exceeds 2^31 entries");
        // lane-mask rows: per target octant, the keys a target has with the eight children of
        // one split source cell get one group of eight positions -- same level: x offset
        // n = 2 (child - target) in half sides, u = n / 2 + (target octant bit), group u >> 1,
        // position u & 1 (the child's bit); finer sources (level difference d > 0): u = (n - 1
        // + (d == 1 ? 2 : 0)) / 2 -- and the keys with coarser sources follow one by one
        // (large key sets, as in deep adaptive trees, keep the plain layout: the host work of
        // the grouping would cost more than it saves)
        int64_t row = nkeys;
        std::vector<int32_t> hpos(8 * (size_t)nkeys);
        bool grouped = false;
        if (nkeys <= kGroupedKeysMax) {
            int64_t rmax = 0;
            std::vector<int32_t> tmp(nkeys);
            std::unordered_map<uint64_t, int32_t> gid;
            gid.reserve(2 * (size_t)nkeys);
            std::vector<int64_t> neg;
            for (int o = 0; o < 8; ++o) {
                gid.clear();
                neg.clear();
                int32_t ng = 0;
                for (int64_t k2 = 0; k2 < nkeys; ++k2) {
                    const uint64_t key = hkeys[k2];
                    const int dl = int(key >> 57) - 32;
                    if (dl < 0) {
                        neg.push_back(k2);
                        continue;
                    }
                    int64_t g3[3];
                    int sub = 0;
                    for (int ax = 0; ax < 3; ++ax) {
                        const int64_t n = int64_t((key >> (38 - 19 * ax)) & 0x7ffff) - kKeyOffBias;
                        const int ob = (o >> (2 - ax)) & 1;
                        const int64_t u = dl == 0 ? n / 2 + ob : (n - 1 + (dl == 1 ? 2 : 0)) / 2;
                        g3[ax] = u >> 1;   // arithmetic shift: floor for negative offsets
                        sub |= int(u & 1) << (2 - ax);
                    }
                    const uint64_t g = pack_key(dl, g3[0], g3[1], g3[2]);
                    auto it = gid.find(g);
                    if (it == gid.end()) it = gid.emplace(g, ng++).first;
                    tmp[k2] = 8 * it->second + sub;
                }
                for (size_t j = 0; j < neg.size(); ++j) tmp[neg[j]] = 8 * ng + (int32_t)j;
                rmax = std::max<int64_t>(rmax, 8 * (int64_t)ng + (int64_t)neg.size());
                std::copy(tmp.begin(), tmp.end(), hpos.begin() + (size_t)o * nkeys);
            }
            // rows much longer than the key count (sparse groups): the plain layout instead
            if (rmax <= 3 * nkeys && ntiles * rmax < (int64_t(1) << 31)) {
                row = rmax;
                grouped = true;
            }
        }
        if (!grouped)
            for (int o = 0; o < 8; ++o)
                for (int64_t k2 = 0; k2 < nkeys; ++k2) hpos[(size_t)o * nkeys + k2] = (int32_t)k2;
        int32_t *lpos = a.get_n<int32_t>(8 * nkeys);
        mb.upload(lpos, hpos.data(), 4 * hpos.size(), s);
        uint8_t *tile_oct = a.get_n<uint8_t>(ntiles);
        {
            std::vector<uint8_t> ho(ntiles);
            for (int b2 = 0; b2 < kBuckets; ++b2)
                for (int64_t t = btile[b2]; t < btile[b2 + 1]; ++t) ho[t] = (uint8_t)(b2 % 8);
            mb.upload(tile_oct, ho.data(), ntiles, s);
        }
        const int64_t nlanes = ntiles * row;
        unsigned long long *lanes = a.get_n<unsigned long long>(nlanes);
        fill_i32(reinterpret_cast<int32_t *>(lanes), 0, 2 * nlanes, s);
        hipLaunchKernelGGL(k_key_ids, std::min(grid1(nm2l), 4096), 256, 0, s, (const int2 *)m2l, nm2l,
                           (const int32_t *)slot_id, (const int32_t *)dsame, (const int32_t *)cell_tile,
                           (const int32_t *)cell_lane, (const uint8_t *)tile_oct, (const int32_t *)lpos, nkeys, row,
                           pkid, lanes, &counts[0]);
        int32_t *present = a.get_n<int32_t>(ntk), *entry_of = a.get_n<int32_t>(ntk + 1);
        // in mixed precision the root tiles stay whole: their FP64 path reads their entries
        const int64_t root_tiles = P->prec == FMM_PREC_MIXED ? btile[(size_t)kRootLevels * 8] : 0;
        int fill_pct = kDenseFillPct;
        if (const char *ev = getenv("FMM_M2L_DENSE_PCT")) fill_pct = std::max(0, std::min(101, atoi(ev)));
        unsigned long long *nsparse = a.get_n<unsigned long long>(1);
        fill_i32(reinterpret_cast<int32_t *>(nsparse), 0, 2, s);
        hipLaunchKernelGGL(k_dense_flags, std::min(grid1(ntk), 4096), 256, 0, s, (const unsigned long long *)lanes,
                           (const uint8_t *)tile_oct, (const int32_t *)lpos, row, ntk, nkeys, fill_pct, root_tiles,
                           present, nsparse);
        int64_t npool = 0;
        {
            const uint64_t t = mb.next_ticket();
            publish(nsparse, 8, mb, t, s);
            mb.wait(t, s);
            npool = (int64_t)mb.data_host<uint64_t>()[0];
        }
        a.put(nsparse);
        // fill_pct above 100 pools every pair and keeps the pool whatever its shape (a test mode)
        const bool force_pool = fill_pct > 100;
        const bool try_pool = npool > 0 && (force_pool || 100 * npool >= (int64_t)kPoolMinPct * nm2l);
        if (npool > 0 && !try_pool) {
            // a small pool is not built: every (tile, key) cell with a pair is an entry
            hipLaunchKernelGGL(k_dense_flags, std::min(grid1(ntk), 4096), 256, 0, s, (const unsigned long long *)lanes,
                               (const uint8_t *)tile_oct, (const int32_t *)lpos, row, ntk, nkeys, 0, (int64_t)0,
                               present, (unsigned long long *)nullptr);
            npool = 0;
        }
        // dense entries (their sources in a first array; the slot entries, if any, follow them)
        int64_t ne_d = exclusive_scan_i32(present, entry_of, ntk, a, s);
        {
            const int32_t tot = (int32_t)ne_d;
            mb.upload(entry_of + ntk, &tot, 4, s);
        }
        int32_t *dsrc = a.get_n<int32_t>(ne_d * kTileN);
        fill_i32(dsrc, -1, ne_d * kTileN, s);
        uint8_t *pool = try_pool ? a.get_n<uint8_t>(nm2l) : nullptr;
        auto fill_entries = [&](int32_t *dst, uint8_t *pl) {
            hipLaunchKernelGGL(k_fill_entries, grid1(nm2l), 256, 0, s, (const int2 *)m2l, nm2l, (const int32_t *)pkid,
                               (const int32_t *)cell_tile, (const int32_t *)cell_lane, (const int32_t *)entry_of,
                               nkeys, dst, pl);
        };
        fill_entries(dsrc, pool);
        SlotTiles st;
        if (try_pool) {
            // ---- slot pool (given up when its slots would tile poorly)
            lg("m2l dense cells");
            build_slots(P, C, pkid, recs, nrec, pool, npool, a, s, st, force_pool);
        }
        if (pool) a.put(pool);
        if (st.ntiles == 0 && npool > 0) {
            // no pool: every (tile, key) cell with a pair is an entry of its target tile
            hipLaunchKernelGGL(k_dense_flags, std::min(grid1(ntk), 4096), 256, 0, s, (const unsigned long long *)lanes,
                               (const uint8_t *)tile_oct, (const int32_t *)lpos, row, ntk, nkeys, 0, (int64_t)0,
                               present, (unsigned long long *)nullptr);
            ne_d = exclusive_scan_i32(present, entry_of, ntk, a, s);
            {
                const int32_t tot = (int32_t)ne_d;
                mb.upload(entry_of + ntk, &tot, 4, s);
            }
            a.put(dsrc);
            dsrc = a.get_n<int32_t>(ne_d * kTileN);
            fill_i32(dsrc, -1, ne_d * kTileN, s);
            fill_entries(dsrc, (uint8_t *)nullptr);
        }
        if (st.ntiles == 0) npool = 0;
        P->npool = npool;
        P->nslots = st.nslots;
        P->nslot_tiles = st.ntiles;
        a.put(lanes);
        a.put(lpos);
        a.put(tile_oct);
        a.put(recs);
        recs = nullptr;
        lg("m2l slot pool");

        const int64_t ne = ne_d + st.ne;
        P->nentries = ne;
        P->entry_key = a.get_n<int32_t>(ne);
        if (st.ne == 0) {
            P->entry_src = dsrc;
        } else {
            P->entry_src = a.get_n<int32_t>(ne * kTileN);
            if (ne_d > 0)
                HIP_CHECK(hipMemcpyAsync(P->entry_src, dsrc, sizeof(int32_t) * ne_d * kTileN, hipMemcpyDeviceToDevice, s));
            fill_i32(P->entry_src + ne_d * kTileN, -1, st.ne * kTileN, s);
            a.put(dsrc);
        }
        hipLaunchKernelGGL(k_entry_keys, grid1(ntk), 256, 0, s, (const int32_t *)present, (const int32_t *)entry_of, ntk,
                           nkeys, P->entry_key);
        if (st.ntiles > 0) {
            hipLaunchKernelGGL(k_slot_entries, grid1(st.nslots), 256, 0, s, (const int32_t *)st.tflag,
                               (const int32_t *)st.tid, (const int32_t *)st.gflag, (const int32_t *)st.gid,
                               (const int32_t *)st.gstart, (const int32_t *)st.sorted, st.nslots,
                               (const int32_t *)st.slot_b0, (const int32_t *)st.slot_ym, (const int32_t *)st.tile_eoff,
                               ne_d, (int64_t)0, P->entry_src, P->slot_pos);
            hipLaunchKernelGGL(k_slot_entry_keys, grid1(st.ntiles), 256, 0, s, (const int32_t *)st.tile_sig,
                               (const int32_t *)st.tile_eoff, st.ntiles, (const int32_t *)st.sig_keys,
                               (const int32_t *)st.sig_n, ne_d, P->entry_key);
        }
        P->entry_mask = a.get_n<uint8_t>(ne);
        int32_t *nsrc = !key_kept.empty() ? a.get_n<int32_t>(ne) : nullptr;
        hipLaunchKernelGGL(k_entry_masks, grid1(ne), 256, 0, s, (const int32_t *)P->entry_src, ne, P->entry_mask, nsrc);
        if (nsrc) {
            // pair-weighted fraction of operator blocks the variable-order M2L applies
            std::vector<int32_t> hn(ne), hk(ne);
            HIP_CHECK(hipMemcpyAsync(hn.data(), nsrc, 4 * ne, hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipMemcpyAsync(hk.data(), P->entry_key, 4 * ne, hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            double num = 0, den = 0, rk = 0;
            for (int64_t e2 = 0; e2 < ne; ++e2) {
                num += (double)hn[e2] * key_kept[hk[e2]];
                den += (double)hn[e2];
                if (!svd_rank.empty()) rk += (double)hn[e2] * svd_rank[hk[e2]];
            }
            P->m2l_kept = den > 0 ? num / den : 1.0;
            P->svd_rank_mean = den > 0 ? rk / den : 0.0;
            a.put(nsrc);
        }
        int32_t *tile_first = a.get_n<int32_t>(ntiles);
        hipLaunchKernelGGL(k_tile_first, grid1(ntiles), 256, 0, s, (const int32_t *)entry_of, ntiles, nkeys, tile_first);
        std::vector<int32_t> htf(ntiles);
        if ((int64_t)(4 * ntiles) <= Mailbox::kFetchBytes) {
            std::memcpy(htf.data(), mb.fetch(tile_first, 4 * ntiles, s), 4 * ntiles);
        } else {
            HIP_CHECK(hipMemcpyAsync(htf.data(), tile_first, 4 * ntiles, hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
        }
        a.put(dsame);
        a.put(table); a.put(slot_id); a.put(dkeys); a.put(present); a.put(entry_of); a.put(pkid);
        a.put(tile_first); a.put(cell_tile); a.put(cell_lane);
        lg("m2l entries");

        // work items: split each tile's entries into pieces so that there are enough items
        // to fill the chip.  Items are ordered piece-major, then by their first operator key:
        // the workgroups in flight work on the same part of the key range (entries are
        // key-sorted inside a tile), so the operators they stream stay in L2.
        htf.push_back((int32_t)ne_d);
        int64_t piece = kEntriesPerWork, items = 4096;   // tuning knobs, overridable from the environment
        if (const char *ev = getenv("FMM_M2L_PIECE")) piece = std::max<int64_t>(1, atoll(ev));
        if (const char *ev = getenv("FMM_M2L_ITEMS")) items = std::max<int64_t>(1, atoll(ev));
        int64_t per = std::max<int64_t>(piece, (ne + items - 1) / items);
        // pieces of each tile: count and size (a tile split in several pieces sums them)
        std::vector<int32_t> npc(ntiles), psz(ntiles);
        int64_t maxp = 0, nitems = 0;
        for (int64_t t = 0; t < ntiles; ++t) {
            const int64_t cntE = htf[t + 1] - htf[t];
            const int64_t chunks = std::max<int64_t>(1, (cntE + per - 1) / per);
            const int64_t sz = std::max<int64_t>(1, (cntE + chunks - 1) / chunks);
            npc[t] = (int32_t)((cntE + sz - 1) / sz);
            psz[t] = (int32_t)sz;
            maxp = std::max<int64_t>(maxp, npc[t]);
            nitems += npc[t];
        }
        std::vector<int4> order;   // piece-major
        order.reserve(nitems);
        for (int64_t k2 = 0; k2 < maxp; ++k2)
            for (int64_t t = root_tiles; t < ntiles; ++t)   // mixed: the root tiles run in FP64 only
                if (k2 < npc[t] && htf[t + 1] > htf[t]) {
                    const int c0 = htf[t] + (int)k2 * psz[t];
                    order.push_back(make_int4((int)t, c0, std::min(htf[t + 1], c0 + psz[t]), npc[t] > 1 ? 1 : 0));
                }
        if ((int64_t)(4 * ne_d) <= Mailbox::kFetchBytes && !order.empty()) {
            // then by the operator key of the first entry (a stable counting sort): tiles of
            // different boundary classes hold different key sets, and the workgroups in
            // flight should stream the same operators
            const int32_t *hk = static_cast<const int32_t *>(mb.fetch(P->entry_key, 4 * ne_d, s));
            std::vector<int32_t> kpos(nkeys + 1, 0);
            for (const int4 &u : order) ++kpos[hk[u.y] + 1];
            for (int64_t k2 = 0; k2 < nkeys; ++k2) kpos[k2 + 1] += kpos[k2];
            std::vector<int4> by_key(order.size());
            for (const int4 &u : order) by_key[kpos[hk[u.y]]++] = u;
            order.swap(by_key);
        }
        if (st.ntiles == 0) {
            // the last quarter of the items, longest first: the final workgroups of the launch
            // are the short ones, so the chip drains evenly (slot tiles, short, come last)
            const size_t k0 = order.size() - order.size() / 4;
            std::stable_sort(order.begin() + k0, order.end(),
                             [](const int4 &u, const int4 &v) { return u.z - u.y > v.z - v.y; });
        }
        // work items in launch order (split pieces numbered in that order), and per tile
        // the indices of its items in launch order
        std::vector<int4> hw(order.size());
        std::vector<int32_t> htw(ntiles + 1, 0), htwi(order.size());
        int64_t nsplit = 0;
        for (size_t i = 0; i < order.size(); ++i) {
            int4 w4 = order[i];
            if (w4.w) w4.w = (int)(++nsplit);
            hw[i] = w4;
            ++htw[w4.x + 1];
        }
        for (int64_t t = 0; t < ntiles; ++t) htw[t + 1] += htw[t];
        {
            std::vector<int32_t> fillp(htw.begin(), htw.end() - 1);
            for (size_t i = 0; i < hw.size(); ++i) htwi[fillp[hw[i].x]++] = (int32_t)i;
        }
        const int64_t nwd = (int64_t)hw.size();
        P->nwork = nwd + st.ntiles;
        P->work = a.get_n<int4>(P->nwork);
        P->tile_work = a.get_n<int32_t>(ntiles + 1);
        P->tile_work_idx = a.get_n<int32_t>(std::max<int64_t>(nwd, 1));
        if (nwd > 0) mb.upload(P->work, hw.data(), sizeof(int4) * hw.size(), s);
        mb.upload(P->tile_work, htw.data(), 4 * (ntiles + 1), s);
        if (nwd > 0) mb.upload(P->tile_work_idx, htwi.data(), 4 * nwd, s);
        // slot tiles: one work item each, after the dense ones, writing partial tiles
        // nsplit .. nsplit + st.ntiles - 1; slot q's column is partial column slot_pos[q]
        if (st.ntiles > 0) {
            hipLaunchKernelGGL(k_slot_work, grid1(st.ntiles), 256, 0, s, (const int32_t *)st.tile_eoff,
                               (const int32_t *)st.tile_ne, st.ntiles, ne_d, nsplit, P->work + nwd);
            hipLaunchKernelGGL(k_shift_pos, grid1(st.nslots), 256, 0, s, P->slot_pos, st.nslots, nsplit * kTileN);
        }
        P->npartial = nsplit + st.ntiles;   // before release(), which clears the counts
        st.release(a);

        // mixed precision: the root levels accumulate in FP64, with FP64 operators for the
        // keys their tiles use and their own split into small work items
        if (P->prec == FMM_PREC_MIXED) {
            const int rl = std::min<int>(kRootLevels, P->max_level + 1);
            P->nroot = P->level_off[rl];
            P->Md = a.get_n<double>(P->nroot * P->KP);
            P->Ld = a.get_n<double>(P->nroot * P->KP);
            const int64_t tr = btile[(size_t)kRootLevels * 8];
            P->ntiles_root = tr;
            if (tr > 0) {
                const int64_t ner = htf[tr];
                std::vector<int32_t> hek(ner);
                HIP_CHECK(hipMemcpyAsync(hek.data(), P->entry_key, 4 * ner, hipMemcpyDeviceToHost, s));
                HIP_CHECK(hipStreamSynchronize(s));
                std::vector<char> used(nkeys, 0);
                for (int32_t kk : hek) used[kk] = 1;
                std::vector<uint64_t> rkeys;
                std::vector<int64_t> rid;
                for (int64_t kk = 0; kk < nkeys; ++kk)
                    if (used[kk]) { rkeys.push_back(hkeys[kk]); rid.push_back(kk); }
                std::vector<uint64_t> rp, all(nkeys, 0);
                m2l_operator_ptrs64(P->p, rkeys, rp);
                for (size_t q2 = 0; q2 < rid.size(); ++q2) all[rid[q2]] = rp[q2];
                uint64_t *d64 = a.get_n<uint64_t>(nkeys);
                mb.upload(d64, all.data(), 8 * nkeys, s);
                P->key_f64 = d64;
                constexpr int64_t kPiece64 = 24;
                std::vector<int4> w64;
                std::vector<int32_t> tw(tr + 1), twi;
                int64_t slot = 0;
                for (int64_t t = 0; t < tr; ++t) {
                    tw[t] = (int32_t)twi.size();
                    const int64_t e0 = htf[t], e1 = htf[t + 1];
                    const bool split = e1 - e0 > kPiece64;
                    for (int64_t c0 = e0; c0 < e1; c0 += kPiece64) {
                        twi.push_back((int32_t)w64.size());
                        w64.push_back(make_int4((int)t, (int)c0, (int)std::min(e1, c0 + kPiece64), split ? (int)(++slot) : 0));
                    }
                }
                tw[tr] = (int32_t)twi.size();
                P->nwork64 = (int64_t)w64.size();
                P->work64 = a.get_n<int4>(P->nwork64);
                P->tile_work64 = a.get_n<int32_t>(tr + 1);
                P->tile_work_idx64 = a.get_n<int32_t>(P->nwork64);
                mb.upload(P->work64, w64.data(), sizeof(int4) * w64.size(), s);
                mb.upload(P->tile_work64, tw.data(), 4 * (tr + 1), s);
                mb.upload(P->tile_work_idx64, twi.data(), 4 * P->nwork64, s);
                if (slot > 0) P->partial64 = a.get_n<double>(slot * kTileN * P->KP);
            }
        }
    }

    if (recs) a.put(recs);   // a plan without M2L pairs
    lg("m2l work items");
    // join the near-field lists built on the side stream
    HIP_CHECK(hipEventRecord(P->ev_join, P->side));
    HIP_CHECK(hipStreamWaitEvent(s, P->ev_join, 0));
    a.put(p2p);
    lg("p2p lists (joined)");
    // ---- evaluation workspace
    const int KP = P->KP;
    P->M = a.get_n<float>(nc * KP);
    P->L = a.get_n<float>(nc * KP);
    if (P->npartial > 0) P->partial = a.get_n<float>(P->npartial * kTileN * KP);
    P->far4 = a.get_n<float4>(n);
    P->near4 = a.get_n<float4>(n);
    if (P->prec == FMM_PREC_MIXED) {
        P->Mh = a.get_n<_Float16>(nc * KP);
        P->Ml = a.get_n<_Float16>(nc * KP);
        P->Msinv = a.get_n<float>(nc);
    }
    {
        const uint64_t t = mb.next_ticket();
        publish(counts, 48, mb, t, s);
        mb.wait(t, s);
        P->nm2l_same = (int64_t)mb.data_host<uint64_t>()[0];
        P->p2p_interactions = (int64_t)mb.data_host<uint64_t>()[1];
        P->nseg = (int64_t)mb.data_host<uint64_t>()[2];
        P->np2p_items = (int64_t)mb.data_host<uint64_t>()[3];
        P->np2p_part = (int64_t)mb.data_host<uint64_t>()[4];
        if (P->nseg >= (int64_t)INT32_MAX) fail(FMM_EUNSUPPORTED, "near-field run count exceeds 2^31");
        if (P->np2p_items >= (int64_t)INT32_MAX) fail(FMM_EUNSUPPORTED, "near-field work items exceed 2^31");
    }
    P->p2p_items = a.get_n<int4>(P->np2p_items);
    hipLaunchKernelGGL(k_p2p_items, grid1(P->nleaves), 256, 0, s, (int64_t)P->nleaves, (const int32_t *)p2p_pieces,
                       (const int32_t *)p2p_item_off, (const int32_t *)p2p_part_off, P->p2p_items);
    if (P->np2p_part > 0) P->p2p_part = a.get_n<float4>(P->np2p_part * kP2PThreads);
    a.put(counts);
    HIP_CHECK(hipStreamSynchronize(s));
    lg("workspace");
    if (getenv("FMM_VALIDATE_PLAN")) validate_m2l(P, s);
}

}  // namespace fmm
