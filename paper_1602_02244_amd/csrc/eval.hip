// Evaluation kernels of the FMM (Sec. 1: upward pass P2M/M2M, M2L over the
// interaction lists, downward pass L2L/L2P, near-field P2P) for CDNA4.
//
// Expansions are scaled complex solid harmonics stored as real vectors (see
// operators.cpp); every cell's coefficients use its own side s as the length unit,
// so one translation matrix serves all levels.
//
//   P2M   one wave per leaf; each lane evaluates R_lm at one body, wave reductions
//   M2M   one wave per parent; lanes own output rows, child vectors broadcast from LDS
//   M2L   grouped GEMM on FP32 MFMA (16x16x4): a tile of 64 target cells (same level,
//         same octant, Morton order) accumulates T_key * [M of the 64 sources] over the
//         tile's operator keys; T streams from L2, the gathered sources sit in LDS
//   L2L   one wave per cell
//   L2P   one wave per leaf; potential and gradient from the local expansion
//   P2P   one 256-thread workgroup per target leaf; source bodies staged through LDS in
//         batches of 1024, each lane owns (target, source subset), rsqrt inner loop
#include <algorithm>
#include <cmath>

#include "fmm_internal.h"

namespace fmm {

template <int P> struct Dims {
    static constexpr int NT = (P + 1) * (P + 2) / 2;    // (l, m >= 0) pairs
    static constexpr int NC = (P + 1) * (P + 1);        // real coefficients
    static constexpr int KP = (NC + 15) / 16 * 16;      // padded
};

// Regular solid harmonics R_lm(x, y, z), m >= 0, streamed to f(l, m, re, im) one column
// (fixed m, increasing l) at a time, so that only the last two values of a column are live.
template <int P, class F>
__device__ __forceinline__ void stream_regular(float x, float y, float z, F &&f) {
    const float r2 = x * x + y * y + z * z;
    float mr = 1.f, mi = 0.f;                   // R_mm
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            const float c = -1.f / (2.f * m);
            const float nr = c * (x * mr - y * mi), ni = c * (x * mi + y * mr);
            mr = nr;
            mi = ni;
        }
        f(m, m, mr, mi);
        if (m < P) {
            float pr = mr, pi = mi;             // R_{l-1,m}
            float cr = z * mr, ci = z * mi;     // R_{m+1,m}
            f(m + 1, m, cr, ci);
#pragma unroll
            for (int l = m + 1; l < P; ++l) {
                const float den = 1.f / (float)((l + m + 1) * (l - m + 1));
                const float c1 = (2 * l + 1) * den;
                const float nr = c1 * z * cr - den * r2 * pr, ni = c1 * z * ci - den * r2 * pi;
                pr = cr;
                pi = ci;
                cr = nr;
                ci = ni;
                f(l + 1, m, cr, ci);
            }
        }
    }
}

// The same stream with the loops kept rolled: for callers that index their coefficients
// at run time (from LDS), where full unrolling only lengthens live ranges.
template <int P, class F>
__device__ __forceinline__ void stream_regular_rolled(float x, float y, float z, F &&f) {
    const float r2 = x * x + y * y + z * z;
    float mr = 1.f, mi = 0.f;                   // R_mm
#pragma unroll 1
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            const float c = -1.f / (2.f * m);
            const float nr = c * (x * mr - y * mi), ni = c * (x * mi + y * mr);
            mr = nr;
            mi = ni;
        }
        f(m, m, mr, mi);
        if (m < P) {
            float pr = mr, pi = mi;             // R_{l-1,m}
            float cr = z * mr, ci = z * mi;     // R_{m+1,m}
            f(m + 1, m, cr, ci);
#pragma unroll 1
            for (int l = m + 1; l < P; ++l) {
                const float den = 1.f / (float)((l + m + 1) * (l - m + 1));
                const float c1 = (2 * l + 1) * den;
                const float nr = c1 * z * cr - den * r2 * pr, ni = c1 * z * ci - den * r2 * pi;
                pr = cr;
                pi = ci;
                cr = nr;
                ci = ni;
                f(l + 1, m, cr, ci);
            }
        }
    }
}

__device__ __forceinline__ void cell_center(int lvl, int ix, int iy, int iz, double x0x, double x0y, double x0z, int k,
                                            double &cx, double &cy, double &cz, double &inv_side) {
    double side = ldexp(1.0, k - lvl);
    inv_side = ldexp(1.0, lvl - k);
    cx = x0x + ((double)ix + 0.5) * side;
    cy = x0y + ((double)iy + 0.5) * side;
    cz = x0z + ((double)iz + 0.5) * side;
}

struct Geo {
    const int32_t *start, *count, *level, *ix, *iy, *iz, *parent, *child0, *nchild;
    double x0x, x0y, x0z;
    int k;
};

// ------------------------------------------------------------------ P2M
// Two leaves per wave, one per half-wave.  Each lane evaluates the harmonics of one
// body (streamed into registers, times its charge); the 32 lanes of a half-wave then
// sum their vectors with a reduce-scatter over cross-lane shuffles (five halving
// steps), after which lane h holds the finished coefficients NF*h .. NF*h + NF - 1.
// No LDS, so occupancy is set by registers alone.
template <int P>
__global__ void __launch_bounds__(64) k_p2m(const int32_t *leaves, int64_t nleaves, Geo g, const float4 *bodies,
                                            float *M) {
    using D = Dims<P>;
    constexpr int NV = (D::NC + 31) / 32 * 32;   // register vector length
    constexpr int NF = NV / 32;                  // coefficients per lane after the reduction
    const int lane = threadIdx.x, half = lane >> 5, hl = lane & 31;
    const int64_t li = 2 * (int64_t)blockIdx.x + half;
    const bool has = li < nleaves;
    const int c = leaves[has ? li : 0];
    const int s = g.start[c], n = has ? g.count[c] : 0;
    double cx, cy, cz, inv;
    cell_center(g.level[c], g.ix[c], g.iy[c], g.iz[c], g.x0x, g.x0y, g.x0z, g.k, cx, cy, cz, inv);
    const int nmax = max(n, __shfl_xor(n, 32, 64));
    float acc[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) acc[i] = 0.f;
    for (int base = 0; base < nmax; base += 32) {
        const int j = base + hl;
        float ux = 0.f, uy = 0.f, uz = 0.f, q = 0.f;
        if (j < n) {
            float4 b = bodies[s + j];
            ux = (float)(((double)b.x - cx) * inv);
            uy = (float)(((double)b.y - cy) * inv);
            uz = (float)(((double)b.z - cz) * inv);
            q = b.w;
        }
        // Mt_lm = sum q conj(R_lm(u))
        float v[NV];
#pragma unroll
        for (int d = D::NC; d < NV; ++d) v[d] = 0.f;
        stream_regular<P>(ux, uy, uz, [&](int l, int m, float re, float im) {
            if (m == 0) {
                v[l * l] = q * re;
            } else {
                v[l * l + 2 * m - 1] = q * re;
                v[l * l + 2 * m] = -q * im;
            }
        });
#pragma unroll
        for (int st = 0; st < 5; ++st) {
            const int o = 16 >> st, H = (NV >> st) / 2;
            const bool upper = (hl & o) != 0;
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const float send = upper ? v[i] : v[i + H];
                const float keep = upper ? v[i + H] : v[i];
                v[i] = keep + __shfl_xor(send, o, 64);
            }
        }
#pragma unroll
        for (int i = 0; i < NF; ++i) acc[i] += v[i];
    }
    if (!has) return;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const int d = NF * hl + i;
        if (d < D::KP) M[(int64_t)c * D::KP + d] = acc[i];
    }
}

// ------------------------------------------------------------------ M2L (FP32 MFMA)
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const floatx4 gfloatx4;   // global-memory float x4

// Workgroup = 4 waves.  Output tile: KP rows x 64 target columns, in 16x16 blocks.
// Wave w owns row blocks w, w+4, ... and all four column blocks.  The K loop runs in
// chunks of 16 coefficients; inside a chunk lane l feeds k = 16*kc + 4*s + l/16 to MFMA
// step s, for both operands: the operators are stored with a 4 x 4 transpose inside
// every 16-wide chunk of columns and the gathered vectors are written to LDS in the same
// order, so each lane still reads its four k as one float4, and a step whose four k are
// all padding (k >= NC, in the last chunk) is not issued.
//
// Software pipeline, with no branch on loaded data so that every wait is a counted one:
//   entry e+2: source indices (lane = column), operator key and column mask are loaded;
//   entry e+1: the operator pointer is resolved, and its 64 gathered source vectors are
//              loaded one k chunk (16 coefficients of every source) per k chunk of entry e
//              (the source index reaches the loading lane by a cross-lane shuffle; empty
//              columns load row 0 and are zeroed when stored to LDS);
//   entry e:   T streams two k chunks ahead of its MFMAs (one when there is a single
//              chunk), and the last chunks prefetch the first ones of entry e+1's operator.
// Column blocks with no source in an entry (mask bit clear; MASKED only) are skipped.
//
// The same kernel runs M2L (all levels at once, split into work items), M2M (per
// level: targets are parents, one entry per child octant) and L2L (per level:
// targets share an octant, the source is the parent; ADD accumulates onto the
// M2L result).
template <int P, bool ADD, bool MASKED, bool VARORD = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P <= 12 ? 2 : 1))) k_gemm(const int4 *work, const int32_t *entry_key, const int32_t *entry_src,
                                              const uint8_t *entry_mask, const uint64_t *key_ptr, const float *M,
                                              float *L, float *partial, const int32_t *tile_targets,
                                              const uint32_t *key_rows = nullptr) {
    using D = Dims<P>;
    constexpr int KP = D::KP;
    constexpr int KPS = KP + 4;                  // LDS row stride (bank spread)
    constexpr int NRB = KP / 16;                 // row blocks
    constexpr int RBW = (NRB + 3) / 4;           // row blocks per wave
    constexpr int NKC = KP / 16;                 // k chunks
    constexpr int NQ = KP / 4;                   // float4 per coefficient vector
    constexpr int NPF = kTileN * NQ / 256;       // gathered float4 per thread per entry
    static_assert(kTileN == 64 && (kTileN * NQ) % 256 == 0 && NPF == NKC && NQ == 4 * NKC,
                  "one gather piece per k chunk");
    __shared__ __attribute__((aligned(16))) float Ms[kTileN * KPS];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar branches
    const int li = lane & 15, lg = lane >> 4;
    const int4 w = work[blockIdx.x];
    const int e0 = w.y, e1 = w.z;
    if (e0 >= e1) return;
    floatx4 acc[RBW][4];
#pragma unroll
    for (int r = 0; r < RBW; ++r)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[r][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    auto clampe = [&](int e) { return min(e, e1 - 1); };
    // gather layout: thread tid copies column tid/4, and piece i is k chunk i (coefficients
    // 16 i .. 16 i + 15, one float4 per thread)
    const int gcol = tid >> 2, gsub = tid & 3;
    float4 pre[NPF];
    int src = -1;
    auto gather_src = [&](int idxv) { src = __shfl(idxv, gcol, 64); };
    auto gather_piece = [&](int i, uint32_t used) {
        // a chunk no row of the operator uses re-reads chunk 0 (cached) instead
        const int q4 = (!VARORD || ((used >> i) & 1u)) ? 4 * i + gsub : gsub;
        pre[i] = reinterpret_cast<const float4 *>(M + (int64_t)max(src, 0) * KP)[q4];
    };
    auto mask_of = [&](int e) { return MASKED ? (int)entry_mask[e] : 15; };

    // variable order: per row block of the wave, the k chunks of the operator that are kept;
    // word NRB of a key holds the union over all its row blocks
    uint32_t rm[RBW], rmn[RBW];
    auto rows_of = [&](int key, uint32_t *dst) {
#pragma unroll
        for (int r = 0; r < RBW; ++r)
            dst[r] = VARORD ? key_rows[(int64_t)key * (NRB + 1) + min(wave + 4 * r, NRB - 1)] : ~0u;
    };
    auto used_of = [&](int key) { return VARORD ? key_rows[(int64_t)key * (NRB + 1) + NRB] : ~0u; };
    // operators are reached through a pointer table: global loads, not flat ones (a flat
    // load also counts against the LDS wait counter).  A chunk the variable order leaves out
    // is not skipped but re-reads chunk 0 (already in cache): no branch around a load, so
    // every wait stays a counted one.
    auto t_chunk_v = [&](const float *T, int kc, const uint32_t *msk, floatx4 *dst) {
        const gfloatx4 *Tg = (const gfloatx4 *)(T);
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
            const int rb = min(wave + 4 * r, NRB - 1);
            const int kk = (!VARORD || ((msk[r] >> kc) & 1u)) ? kc : 0;
            dst[r] = Tg[((rb * 16 + li) * KP + kk * 16 + 4 * lg) / 4];
        }
    };

    // prologue: entry e0's sources and operator chunk 0; entry e0+1's indices, key and mask
    const int key0 = entry_key[e0];
    gather_src(entry_src[(int64_t)e0 * kTileN + lane]);
    {
        const uint32_t used0 = used_of(key0);
#pragma unroll
        for (int i = 0; i < NPF; ++i) gather_piece(i, used0);
    }
    const float *Tc = reinterpret_cast<const float *>(key_ptr[key0]);
    rows_of(key0, rm);
    int mask = mask_of(e0);
    constexpr bool T2 = NKC >= 2;   // the operator streams two k chunks ahead of its MFMAs
    floatx4 a[RBW], an[RBW], ann[RBW];
#pragma unroll
    for (int r = 0; r < RBW; ++r) a[r] = an[r] = ann[r] = floatx4{0.f, 0.f, 0.f, 0.f};
    t_chunk_v(Tc, 0, rm, a);
    if (T2) t_chunk_v(Tc, 1, rm, an);
    int idx = entry_src[(int64_t)clampe(e0 + 1) * kTileN + lane];
    int key_n = entry_key[clampe(e0 + 1)];
    int mask_n = mask_of(clampe(e0 + 1));

    for (int e = e0; e < e1; ++e) {
        // everything loaded during the previous entry is consumed here, before new loads
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NPF; ++i) {
            // coefficients 16 i + 4 gsub + j go to positions 16 i + 4 j + gsub
            const float4 v = src >= 0 ? pre[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            float *row = &Ms[gcol * KPS + 16 * i + gsub];
            row[0] = v.x;
            row[4] = v.y;
            row[8] = v.z;
            row[12] = v.w;
        }
        gather_src(idx);                         // entry e+1
        const int m = __builtin_amdgcn_readfirstlane(mask);
        const int kn = __builtin_amdgcn_readfirstlane(key_n);
        mask = mask_n;
        __syncthreads();
        // next entry's operator; the entry after that: indices, key, mask
        const float *Tn = reinterpret_cast<const float *>(key_ptr[kn]);
        rows_of(kn, rmn);
        const uint32_t used_n = used_of(kn);
        idx = entry_src[(int64_t)clampe(e + 2) * kTileN + lane];
        key_n = entry_key[clampe(e + 2)];
        mask_n = mask_of(clampe(e + 2));
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
            if (T2) {
                if (kc + 2 < NKC) t_chunk_v(Tc, kc + 2, rm, ann);
                else t_chunk_v(Tn, kc + 2 - NKC, rmn, ann);
            } else {
                if (kc + 1 < NKC) t_chunk_v(Tc, kc + 1, rm, an);
                else t_chunk_v(Tn, 0, rmn, an);
            }
            gather_piece(kc, used_n);            // entry e+1 (a repeat of the last entry at the end)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                if (!((m >> cb) & 1)) continue;
                const float4 b = *reinterpret_cast<const float4 *>(&Ms[(cb * 16 + li) * KPS + kc * 16 + 4 * lg]);
#pragma unroll
                for (int r = 0; r < RBW; ++r) {
                    if (NRB % 4 != 0 && wave + 4 * r >= NRB) continue;
                    if (VARORD && !((rm[r] >> kc) & 1u)) continue;
                    // step s covers k = 16 kc + 4 s .. 16 kc + 4 s + 3 (step 0 always holds a real k)
                    acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x, b.x, acc[r][cb], 0, 0, 0);
                    if (16 * kc + 4 < D::NC)
                        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].y, b.y, acc[r][cb], 0, 0, 0);
                    if (16 * kc + 8 < D::NC)
                        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].z, b.z, acc[r][cb], 0, 0, 0);
                    if (16 * kc + 12 < D::NC)
                        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].w, b.w, acc[r][cb], 0, 0, 0);
                }
            }
#pragma unroll
            for (int r = 0; r < RBW; ++r) {
                a[r] = an[r];
                if (T2) an[r] = ann[r];
            }
        }
        Tc = Tn;
#pragma unroll
        for (int r = 0; r < RBW; ++r) rm[r] = rmn[r];
    }
    // output: lane holds D[4*lg + v][li] of each 16x16 block
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
        const int rb = wave + 4 * r;
        if (rb >= NRB) continue;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int col = cb * 16 + li;
            float *dst;
            if (w.w == 0) {
                const int t = tile_targets[(int64_t)w.x * kTileN + col];
                if (t < 0) continue;
                dst = L + (int64_t)t * KP;
            } else {
                dst = partial + ((int64_t)(w.w - 1) * kTileN + col) * KP;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (ADD && w.w == 0) dst[rb * 16 + 4 * lg + v] += acc[r][cb][v];
                else dst[rb * 16 + 4 * lg + v] = acc[r][cb][v];
            }
        }
    }
}

// ------------------------------------------------------------------ M2L, SVD-compressed operators
// The same work items, tiles and entries as k_gemm; every key's operator is applied in
// factored form, A ~ Pf Qf with rank rp (a multiple of 16): per entry Y = Qf Ms (rp x 64,
// k over the KP coefficients), then acc += Pf Y (k over the rank).  Workgroup = 4 waves; in
// the first product wave w computes column block w of Y for every row block, in the second
// it owns output row blocks w, w+4, ... as in k_gemm.  Ms (the gathered source vectors) and
// then Y share one LDS buffer.  The next entry's source vectors are loaded into registers
// while the second product runs (every load is consumed before the next is issued).
template <int P>
__global__ void __launch_bounds__(256) k_gemm_svd(const int4 *work, const int32_t *entry_key, const int32_t *entry_src,
                                                  const uint8_t *entry_mask, const uint64_t *key_svd,
                                                  const int32_t *key_rank, const float *M, float *L, float *partial,
                                                  const int32_t *tile_targets) {
    using D = Dims<P>;
    constexpr int KP = D::KP;
    constexpr int KPS = KP + 4;                  // LDS row stride
    constexpr int NRB = KP / 16;                 // row blocks of the output (and of Y at full rank)
    constexpr int RBW = (NRB + 3) / 4;           // output row blocks per wave
    constexpr int NKC = KP / 16;                 // k chunks of the first product
    static_assert(kTileN == 64, "four 16-column blocks");
    __shared__ __attribute__((aligned(16))) float Ms[kTileN * KPS];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lg = lane >> 4;
    const int4 w = work[blockIdx.x];
    const int e0 = w.y, e1 = w.z;
    if (e0 >= e1) return;
    floatx4 acc[RBW][4];
#pragma unroll
    for (int r = 0; r < RBW; ++r)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[r][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int gcol = tid >> 2, gsub = tid & 3;
    // source vectors of the current entry, in registers until they are stored to LDS
    float4 pre[NKC];
    int src = entry_src[(int64_t)e0 * kTileN + gcol];
    auto gather = [&](int sv) {
#pragma unroll
        for (int i = 0; i < NKC; ++i) pre[i] = reinterpret_cast<const float4 *>(M + (int64_t)max(sv, 0) * KP)[4 * i + gsub];
    };
    gather(src);
    for (int e = e0; e < e1; ++e) {
        const int key = __builtin_amdgcn_readfirstlane(entry_key[e]);
        const int rp = __builtin_amdgcn_readfirstlane(key_rank[key]);
        const int m = __builtin_amdgcn_readfirstlane((int)entry_mask[e]);
        const gfloatx4 *Qg = (const gfloatx4 *)reinterpret_cast<const float *>(key_svd[2 * key]);
        const gfloatx4 *Pg = (const gfloatx4 *)reinterpret_cast<const float *>(key_svd[2 * key + 1]);
        const int src_next = entry_src[(int64_t)min(e + 1, e1 - 1) * kTileN + gcol];
        __syncthreads();   // the previous entry is done with the buffer
#pragma unroll
        for (int i = 0; i < NKC; ++i) {
            // coefficients 16 i + 4 gsub + j go to positions 16 i + 4 j + gsub
            const float4 v = src >= 0 ? pre[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            float *row = &Ms[gcol * KPS + 16 * i + gsub];
            row[0] = v.x;
            row[4] = v.y;
            row[8] = v.z;
            row[12] = v.w;
        }
        src = src_next;
        __syncthreads();
        // first product: column block `wave` of Y for every row block below rp
        const int nrb = rp / 16;
        floatx4 y[NRB];
#pragma unroll
        for (int r = 0; r < NRB; ++r) y[r] = floatx4{0.f, 0.f, 0.f, 0.f};
        const bool mine = (m >> wave) & 1;
        if (mine) {
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) {
                const float4 b = *reinterpret_cast<const float4 *>(&Ms[(wave * 16 + li) * KPS + kc * 16 + 4 * lg]);
#pragma unroll
                for (int r = 0; r < NRB; ++r) {
                    if (r >= nrb) break;
                    const floatx4 a = Qg[((r * 16 + li) * KP + kc * 16 + 4 * lg) / 4];
                    y[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, y[r], 0, 0, 0);
                    if (16 * kc + 4 < D::NC) y[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, y[r], 0, 0, 0);
                    if (16 * kc + 8 < D::NC) y[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, y[r], 0, 0, 0);
                    if (16 * kc + 12 < D::NC) y[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, y[r], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // every wave is done reading Ms
        // Y into the buffer, in the transposed-chunk order of a B operand: column c of Y is
        // buffer row c, rank index k at position 16 (k / 16) + 4 (k % 4) + (k % 16) / 4
#pragma unroll
        for (int r = 0; r < NRB; ++r) {
            if (r >= nrb) break;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = r * 16 + 4 * lg + v;
                Ms[(wave * 16 + li) * KPS + 16 * (k / 16) + 4 * (k % 4) + (k % 16) / 4] = y[r][v];
            }
        }
        __syncthreads();
        gather(src);   // the next entry's sources (a repeat of the last entry's at the end)
        // second product: acc (KP x 64) += Pf (KP x rp) Y (rp x 64)
        for (int kc = 0; kc < nrb; ++kc) {
            floatx4 a[RBW];
#pragma unroll
            for (int r = 0; r < RBW; ++r) {
                const int rb = min(wave + 4 * r, NRB - 1);
                a[r] = Pg[((rb * 16 + li) * rp + kc * 16 + 4 * lg) / 4];
            }
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                if (!((m >> cb) & 1)) continue;
                const float4 b = *reinterpret_cast<const float4 *>(&Ms[(cb * 16 + li) * KPS + kc * 16 + 4 * lg]);
#pragma unroll
                for (int r = 0; r < RBW; ++r) {
                    if (NRB % 4 != 0 && wave + 4 * r >= NRB) continue;
                    acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x, b.x, acc[r][cb], 0, 0, 0);
                    acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].y, b.y, acc[r][cb], 0, 0, 0);
                    acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].z, b.z, acc[r][cb], 0, 0, 0);
                    acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].w, b.w, acc[r][cb], 0, 0, 0);
                }
            }
        }
    }
    // output: lane holds D[4*lg + v][li] of each 16x16 block
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
        const int rb = wave + 4 * r;
        if (rb >= NRB) continue;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int col = cb * 16 + li;
            float *dst;
            if (w.w == 0) {
                const int t = tile_targets[(int64_t)w.x * kTileN + col];
                if (t < 0) continue;
                dst = L + (int64_t)t * KP;
            } else {
                dst = partial + ((int64_t)(w.w - 1) * kTileN + col) * KP;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[rb * 16 + 4 * lg + v] = acc[r][cb][v];
        }
    }
}

// ------------------------------------------------------------------ M2L, split FP16 on MFMA
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));

// Once per evaluation: every cell's multipole vector, normalised by nu (|nu_lm R_lm| <= 1)
// and by a power of two per cell (largest value in [1, 2)), split into FP16 hi + lo.
template <int P>
__global__ void __launch_bounds__(64) k_split_m(const float *M, const float *nu, _Float16 *Mh, _Float16 *Ml,
                                                float *sinv) {
    using D = Dims<P>;
    constexpr int KP = D::KP;
    constexpr int NR = (KP + 63) / 64;
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x;
    float v[NR];
    float m = 0.f;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int d = r * 64 + lane;
        v[r] = d < KP ? M[c * KP + d] * nu[d] : 0.f;
        m = fmaxf(m, fabsf(v[r]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    const float sc = m > 0.f ? exp2f(-floorf(log2f(m))) : 1.f;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int d = r * 64 + lane;
        if (d < KP) {
            const float x = v[r] * sc;
            const _Float16 h = (_Float16)x;
            Mh[c * KP + d] = h;
            Ml[c * KP + d] = (_Float16)(x - (float)h);
        }
    }
    if (lane == 0) sinv[c] = 1.f / sc;
}

// Mixed-precision M2L.  Each operator is stored as diag(rs) (H + Lo) acting on the
// normalised multipoles (H, Lo in FP16, rs powers of two).  Per entry the split
// multipoles of the 64 sources are copied to LDS, the product is taken as
// H hi + H lo + Lo hi on v_mfma_f32_16x16x32_f16 with FP32 accumulation, and the entry's
// result is scaled back (rows by rs, columns by the source's inverse scale) and added in
// FP32.  Tiling, work items, outputs and the software pipeline (indices two entries
// ahead, gathered sources one entry ahead spread over the k steps, operator one k step
// ahead, global loads only) are those of k_gemm, with NW waves: at 11 <= p <= 15 eight,
// so that the row blocks and gather pieces of a wave fit two waves per SIMD (four waves
// would hold one per SIMD).  Every output element sums the same terms in the same
// order whatever NW is.
template <int P>
constexpr int f16_waves() {   // waves per workgroup of k_m2l_f16: 8 fit two waves per SIMD for 11 <= p <= 15
    return P >= 11 && P <= 15 ? 8 : 4;
}

template <int P, int NW = f16_waves<P>()>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(P <= 10 || NW == 8 ? 2 : 1))) k_m2l_f16(const int4 *work, const int32_t *entry_key, const int32_t *entry_src,
                                                 const uint8_t *entry_mask, const uint64_t *key_ptr,
                                                 const _Float16 *Mh, const _Float16 *Ml, const float *sinv, float *L,
                                                 float *partial, const int32_t *tile_targets) {
    using D = Dims<P>;
    constexpr int KP = D::KP;
    constexpr int KPH = KP + 8;                  // LDS row stride in halves
    constexpr int NRB = KP / 16;
    constexpr int NT = 64 * NW;                  // threads
    constexpr int RBW = (NRB + NW - 1) / NW;     // row blocks per wave (wave w: w, w + NW, ...)
    constexpr int NK32 = KP / 32;                // k steps of 32
    constexpr bool TAIL16 = (KP % 32) != 0;      // one k step of 16 at the end
    constexpr int NKS = NK32 + (TAIL16 ? 1 : 0); // k steps
    constexpr int NQ = KP / 8;                   // 16-byte pieces (8 halves) per vector
    constexpr int NG = kTileN * NQ;              // pieces per entry and half
    constexpr int NPF = (NG + NT - 1) / NT;
    static_assert(kTileN == 64, "64-column tiles");
    __shared__ __attribute__((aligned(16))) _Float16 Bh[kTileN * KPH];
    __shared__ __attribute__((aligned(16))) _Float16 Bl[kTileN * KPH];
    __shared__ float colinv[kTileN];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lg = lane >> 4;
    const int4 w = work[blockIdx.x];
    const int e0 = w.y, e1 = w.z;
    if (e0 >= e1) return;
    floatx4 acc[RBW][4];
#pragma unroll
    for (int r = 0; r < RBW; ++r)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[r][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    typedef __attribute__((address_space(1))) const half8 ghalf8;
    typedef __attribute__((address_space(1))) const half4 ghalf4;
    typedef __attribute__((address_space(1))) const float gfloat;
    auto clampe = [&](int e) { return min(e, e1 - 1); };
    auto mask_of = [&](int e) { return (int)entry_mask[e]; };
    half8 ah[RBW], al[RBW], nh[RBW], nl[RBW];
    auto t_step = [&](const _Float16 *H, int kc, half8 *dh, half8 *dl) {   // one 32-wide k step
        const ghalf8 *Hg = (const ghalf8 *)H, *Lg = (const ghalf8 *)(H + KP * KP);
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
            const int rb = min(wave + NW * r, NRB - 1);
            const int off = ((rb * 16 + li) * KP + kc * 32 + 8 * lg) / 8;
            dh[r] = Hg[off];
            dl[r] = Lg[off];
        }
    };
    float4 ph[NPF], pl[NPF];
    int srcs[NPF];
    float pinv = 0.f;
    int csrc = -1;                               // this lane's column source (wave 0)
    auto gather_src = [&](int idxv) {
#pragma unroll
        for (int i = 0; i < NPF; ++i) srcs[i] = __shfl(idxv, min(tid + NT * i, NG - 1) / NQ, 64);
        csrc = idxv;
    };
    auto gather_piece = [&](int i) {
        const int q = min(tid + NT * i, NG - 1) % NQ;
        const int64_t row = (int64_t)max(srcs[i], 0) * KP;
        ph[i] = reinterpret_cast<const float4 *>(Mh + row)[q];
        pl[i] = reinterpret_cast<const float4 *>(Ml + row)[q];
    };
    auto gather_step = [&](int ks) {             // the pieces issued during k step ks
#pragma unroll
        for (int i = ks * NPF / NKS; i < (ks + 1) * NPF / NKS; ++i) gather_piece(i);
        if (ks == 0) pinv = sinv[max(csrc, 0)];
    };

    // prologue
    gather_src(entry_src[(int64_t)e0 * kTileN + lane]);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) gather_step(ks);
    const char *Tc = reinterpret_cast<const char *>(key_ptr[entry_key[e0]]);
    int mask = mask_of(e0);
    if (NK32 > 0) t_step(reinterpret_cast<const _Float16 *>(Tc), 0, ah, al);
    int idx = entry_src[(int64_t)clampe(e0 + 1) * kTileN + lane];
    int key_n = entry_key[clampe(e0 + 1)];
    int mask_n = mask_of(clampe(e0 + 1));

    for (int e = e0; e < e1; ++e) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NPF; ++i) {
            const int g = tid + NT * i;
            if (g < NG) {
                const int col = g / NQ, q = g % NQ;
                const bool ok = srcs[i] >= 0;
                *reinterpret_cast<float4 *>(&Bh[col * KPH + 8 * q]) = ok ? ph[i] : make_float4(0.f, 0.f, 0.f, 0.f);
                *reinterpret_cast<float4 *>(&Bl[col * KPH + 8 * q]) = ok ? pl[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        if (tid < kTileN) colinv[tid] = csrc >= 0 ? pinv : 0.f;
        gather_src(idx);                         // entry e+1
        const int m = __builtin_amdgcn_readfirstlane(mask);
        const int kn = __builtin_amdgcn_readfirstlane(key_n);
        mask = mask_n;
        __syncthreads();
        const _Float16 *H = reinterpret_cast<const _Float16 *>(Tc);
        const char *Tn = reinterpret_cast<const char *>(key_ptr[kn]);
        float4 r4[RBW];                          // this entry's row scales
        {
            const gfloat *rs = (const gfloat *)(H + 2 * KP * KP);
#pragma unroll
            for (int r = 0; r < RBW; ++r) {
                const int rb = min(wave + NW * r, NRB - 1);
                r4[r] = make_float4(rs[rb * 16 + 4 * lg], rs[rb * 16 + 4 * lg + 1], rs[rb * 16 + 4 * lg + 2],
                                    rs[rb * 16 + 4 * lg + 3]);
            }
        }
        idx = entry_src[(int64_t)clampe(e + 2) * kTileN + lane];
        key_n = entry_key[clampe(e + 2)];
        mask_n = mask_of(clampe(e + 2));
        floatx4 tmp[RBW][4];
#pragma unroll
        for (int r = 0; r < RBW; ++r)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) tmp[r][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
        constexpr int k0 = NK32 * 32;
        half4 th[RBW], tl[RBW];
        auto t_tail = [&]() {
            const ghalf4 *Hg = (const ghalf4 *)H, *Lg = (const ghalf4 *)(H + KP * KP);
#pragma unroll
            for (int r = 0; r < RBW; ++r) {
                const int rb = min(wave + NW * r, NRB - 1);
                const int off = ((rb * 16 + li) * KP + k0 + 4 * lg) / 4;
                th[r] = Hg[off];
                tl[r] = Lg[off];
            }
        };
        if (TAIL16 && NK32 == 0) t_tail();
#pragma unroll
        for (int kc = 0; kc < NK32; ++kc) {
            if (kc + 1 < NK32) t_step(H, kc + 1, nh, nl);
            else if (TAIL16) t_tail();
            else t_step(reinterpret_cast<const _Float16 *>(Tn), 0, nh, nl);
            gather_step(kc);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                if (!((m >> cb) & 1)) continue;
                const int boff = (cb * 16 + li) * KPH + kc * 32 + 8 * lg;
                const half8 bh = *reinterpret_cast<const half8 *>(&Bh[boff]);
                const half8 bl = *reinterpret_cast<const half8 *>(&Bl[boff]);
#pragma unroll
                for (int r = 0; r < RBW; ++r) {
                    if (NRB % NW != 0 && wave + NW * r >= NRB) continue;
                    tmp[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[r], bh, tmp[r][cb], 0, 0, 0);
                    tmp[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[r], bl, tmp[r][cb], 0, 0, 0);
                    tmp[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[r], bh, tmp[r][cb], 0, 0, 0);
                }
            }
            if (kc + 1 < NK32 || !TAIL16) {
#pragma unroll
                for (int r = 0; r < RBW; ++r) {
                    ah[r] = nh[r];
                    al[r] = nl[r];
                }
            }
        }
        if (TAIL16) {
            if (NK32 > 0) t_step(reinterpret_cast<const _Float16 *>(Tn), 0, ah, al);
            gather_step(NKS - 1);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                if (!((m >> cb) & 1)) continue;
                const int boff = (cb * 16 + li) * KPH + k0 + 4 * lg;
                const half4 bh = *reinterpret_cast<const half4 *>(&Bh[boff]);
                const half4 bl = *reinterpret_cast<const half4 *>(&Bl[boff]);
#pragma unroll
                for (int r = 0; r < RBW; ++r) {
                    if (NRB % NW != 0 && wave + NW * r >= NRB) continue;
                    tmp[r][cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(th[r], bh, tmp[r][cb], 0, 0, 0);
                    tmp[r][cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(th[r], bl, tmp[r][cb], 0, 0, 0);
                    tmp[r][cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(tl[r], bh, tmp[r][cb], 0, 0, 0);
                }
            }
        }
        // back to the FP32 basis: rows by rs, columns by the source's inverse scale
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
            if (NRB % NW != 0 && wave + NW * r >= NRB) continue;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                if (!((m >> cb) & 1)) continue;
                const float ci = colinv[cb * 16 + li];
                acc[r][cb][0] += r4[r].x * ci * tmp[r][cb][0];
                acc[r][cb][1] += r4[r].y * ci * tmp[r][cb][1];
                acc[r][cb][2] += r4[r].z * ci * tmp[r][cb][2];
                acc[r][cb][3] += r4[r].w * ci * tmp[r][cb][3];
            }
        }
        Tc = Tn;
    }
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
        const int rb = wave + NW * r;
        if (rb >= NRB) continue;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int col = cb * 16 + li;
            float *dst;
            if (w.w == 0) {
                const int t = tile_targets[(int64_t)w.x * kTileN + col];
                if (t < 0) continue;
                dst = L + (int64_t)t * KP;
            } else {
                dst = partial + ((int64_t)(w.w - 1) * kTileN + col) * KP;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[rb * 16 + 4 * lg + v] = acc[r][cb][v];
        }
    }
}

// Sum of a split tile's partial results.  Grid (tile, element chunk); the tile's partial
// slots are read once into LDS.
constexpr int kReduceChunks = 8;
__global__ void __launch_bounds__(256) k_m2l_reduce(int64_t ntiles, const int32_t *tile_work,
                                                    const int32_t *tile_work_idx, const int4 *work,
                                                    const float *partial, const int32_t *tile_targets, int KP,
                                                    float *L) {
    constexpr int kMaxSlots = 256;
    __shared__ int slot[kMaxSlots];
    const int64_t t = blockIdx.x;
    const int w0 = tile_work[t], w1 = tile_work[t + 1];
    const int ns = w1 - w0;
    if (ns < 2) return;
    for (int i = threadIdx.x; i < ns && i < kMaxSlots; i += blockDim.x) slot[i] = work[tile_work_idx[w0 + i]].w - 1;
    __syncthreads();
    const int total = kTileN * KP, per = (total + kReduceChunks - 1) / kReduceChunks;
    const int i0 = blockIdx.y * per, i1 = min(total, i0 + per);
    for (int idx = i0 + threadIdx.x; idx < i1; idx += blockDim.x) {
        const int col = idx / KP, row = idx % KP;
        const int tg = tile_targets[t * kTileN + col];
        if (tg < 0) continue;
        float s = 0.f;
        for (int q = 0; q < ns; ++q) {
            const int sl = q < kMaxSlots ? slot[q] : work[tile_work_idx[w0 + q]].w - 1;
            s += partial[((int64_t)sl * kTileN + col) * KP + row];
        }
        L[(int64_t)tg * KP + row] = s;
    }
}

// Slot pool: every target with slots adds the partial columns of its slots.  One workgroup
// per run of slots of one target: the run is dealt to G groups of KP/4 threads (slot q to
// group (q - q0) mod G, float4 per thread), each group sums its slots in slot order, and the
// G group sums are added to L in group order -- a fixed order, so the result does not
// depend on the schedule.
__global__ void __launch_bounds__(256) k_slot_reduce(int64_t nruns, const int32_t *run_first, const int32_t *run_tgt,
                                                     const int64_t *slot_pos, const float *partial, int KP, float *L) {
    __shared__ float4 part[256];
    const int NQ = KP / 4, G = min(256 / NQ, 16);
    const int g = threadIdx.x / NQ, c = threadIdx.x % NQ;
    for (int64_t r = blockIdx.x; r < nruns; r += gridDim.x) {
        const int q0 = run_first[r], q1 = run_first[r + 1];
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        // group g sums the columns q0 + g, q0 + g + G, ... in that order; eight of them are
        // loaded before they are added, so that their latencies overlap
        constexpr int U = 8;
        if (g < G)
            for (int q = q0 + g; q < q1; q += U * G) {
                float4 v[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (q + u * G < q1) v[u] = reinterpret_cast<const float4 *>(partial + slot_pos[q + u * G] * KP)[c];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (q + u * G < q1) {
                        acc.x += v[u].x;
                        acc.y += v[u].y;
                        acc.z += v[u].z;
                        acc.w += v[u].w;
                    }
            }
        if (g < G) part[g * NQ + c] = acc;
        __syncthreads();
        if (threadIdx.x < NQ) {
            float4 *dst = reinterpret_cast<float4 *>(L + (int64_t)run_tgt[r] * KP) + c;
            float4 sum = *dst;
            for (int h = 0; h < G; ++h) {
                const float4 v = part[h * NQ + c];
                sum.x += v.x;
                sum.y += v.y;
                sum.z += v.z;
                sum.w += v.w;
            }
            *dst = sum;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ FP64 root levels (mixed precision)
// Cells [0, nroot) are the cells of the root levels (cells are numbered level by level).
// Their multipole and local coefficients are accumulated in FP64 (Md, Ld) by one tiled
// FP64 GEMM kernel, with FP64 operators stored transposed ([KP in][KP out]); it serves
// the root M2M (targets: parents, entries: child octants), the root M2L (targets: root
// cells of the M2L tiles) and the root L2L (targets: same-octant cells, source: parent;
// ADD accumulates onto the M2L result).  A source below the root levels is read from
// the FP32 array and widened.
// Grid (work items, row slabs): a workgroup computes the 32-row slab blockIdx.y of the
// KP x 64 output tile, so every tile is spread over KP/32 workgroups.  Thread
// (rt = tid % 8, ct = tid / 8) owns rows 4 rt .. 4 rt + 3 of the slab and columns
// 2 ct, 2 ct + 1.  The entry's 64 source vectors sit in LDS as [k][col].
constexpr int kSlab64 = 32;
template <int P, bool ADD>
__global__ void __launch_bounds__(256) k_gemm64(const int4 *work, const int32_t *entry_key, const int32_t *entry_src,
                                                const uint64_t *key_ptr64, int64_t nroot, const float *in32,
                                                const double *in64, double *out, double *partial,
                                                const int32_t *tile_targets) {
    using D = Dims<P>;
    constexpr int KP = D::KP;
    __shared__ __attribute__((aligned(16))) double B[KP * kTileN];   // [k][col]
    const int tid = threadIdx.x, rt = tid & 7, ct = tid >> 3;
    const int r0 = blockIdx.y * kSlab64 + rt * 4;
    const bool rows_ok = r0 < KP;                // KP is a multiple of 16, so 4-row groups are whole
    const int4 w = work[blockIdx.x];
    double acc[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v][0] = acc[v][1] = 0.0;
    for (int e = w.y; e < w.z; ++e) {
        __syncthreads();
        for (int idx = tid; idx < kTileN * KP; idx += 256) {
            const int col = idx / KP, k = idx % KP;
            const int src = entry_src[(int64_t)e * kTileN + col];
            double v = 0.0;
            if (src >= 0) v = src < nroot ? in64[(int64_t)src * KP + k] : (double)in32[(int64_t)src * KP + k];
            B[k * kTileN + col] = v;
        }
        __syncthreads();
        if (!rows_ok) continue;
        const double *T = reinterpret_cast<const double *>(key_ptr64[entry_key[e]]);
        for (int k = 0; k < D::NC; ++k) {
            const double2 b = *reinterpret_cast<const double2 *>(&B[k * kTileN + ct * 2]);
            const double4 a = *reinterpret_cast<const double4 *>(T + (int64_t)k * KP + r0);
            acc[0][0] += a.x * b.x; acc[0][1] += a.x * b.y;
            acc[1][0] += a.y * b.x; acc[1][1] += a.y * b.y;
            acc[2][0] += a.z * b.x; acc[2][1] += a.z * b.y;
            acc[3][0] += a.w * b.x; acc[3][1] += a.w * b.y;
        }
    }
    if (!rows_ok) return;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int col = ct * 2 + c;
        double *dst;
        if (w.w == 0) {
            const int t = tile_targets[(int64_t)w.x * kTileN + col];
            if (t < 0) continue;
            dst = out + (int64_t)t * KP;
        } else {
            dst = partial + ((int64_t)(w.w - 1) * kTileN + col) * KP;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (ADD && w.w == 0) dst[r0 + v] += acc[v][c];
            else dst[r0 + v] = acc[v][c];
        }
    }
}

__global__ void k_m2l64_reduce(int64_t ntiles, const int32_t *tile_work, const int32_t *tile_work_idx, const int4 *work,
                               const double *partial, const int32_t *tile_targets, int KP, double *Ld) {
    const int64_t t = blockIdx.x;
    const int w0 = tile_work[t], w1 = tile_work[t + 1];
    if (w1 - w0 < 2) return;
    for (int idx = blockIdx.y * blockDim.x + threadIdx.x; idx < kTileN * KP; idx += gridDim.y * blockDim.x) {
        const int col = idx / KP, row = idx % KP;
        const int tg = tile_targets[t * kTileN + col];
        if (tg < 0) continue;
        double s = 0.0;
        for (int wi = w0; wi < w1; ++wi)
            s += partial[((int64_t)(work[tile_work_idx[wi]].w - 1) * kTileN + col) * KP + row];
        Ld[(int64_t)tg * KP + row] = s;
    }
}

// Root leaves take their FP32 P2M result into Md (before the root M2M).
__global__ void k_root_leaves_to64(int64_t nroot, int KP, const int32_t *nchild, const float *M, double *Md) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nroot * KP; i += (int64_t)gridDim.x * blockDim.x)
        if (nchild[i / KP] == 0) Md[i] = (double)M[i];
}

// FP32 copies of the root cells' FP64 coefficients.
__global__ void k_root_to32(int64_t nroot, int KP, const double *in, float *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nroot * KP; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

// ------------------------------------------------------------------ L2P
// Local coefficient (j, m) of a packed real vector, m >= -1: L_{j,-1} = -conj(L_{j,1}).
__device__ __forceinline__ float loc_re(const float *v, int j, int m) {
    if (m > j) return 0.f;
    if (m == 0) return v[j * j];
    if (m > 0) return v[j * j + 2 * m - 1];
    return -v[j * j + 1];
}
__device__ __forceinline__ float loc_im(const float *v, int j, int m) {
    if (m > j || m == 0) return 0.f;
    if (m > 0) return v[j * j + 2 * m];
    return v[j * j + 2];
}

// The term (l, m) of a local expansion at one point (R_lm = rr + i ri): the potential, and
// the gradient through the local expansion of the gradient, whose coefficients of degree l
// come from those of degree l+1: x: (L_{l+1,m-1} - L_{l+1,m+1})/2, y: i (L_{l+1,m+1} +
// L_{l+1,m-1})/2, z: L_{l+1,m}.
template <int P>
__device__ __forceinline__ void l2p_term(const float *v, int l, int m, float rr, float ri, float &f, float &gx,
                                         float &gy, float &gz) {
    const float wgt = m == 0 ? 1.f : 2.f;
    f += wgt * (loc_re(v, l, m) * rr + loc_im(v, l, m) * ri);
    if (l < P) {
        const float zr = loc_re(v, l + 1, m), zi = loc_im(v, l + 1, m);
        const float pr = loc_re(v, l + 1, m + 1), pi = loc_im(v, l + 1, m + 1);
        const float mr = loc_re(v, l + 1, m - 1), mi = loc_im(v, l + 1, m - 1);
        const float xr = 0.5f * (mr - pr), xi = 0.5f * (mi - pi);
        const float yr = -0.5f * (pi + mi), yi = 0.5f * (pr + mr);
        gx += wgt * (xr * rr + xi * ri);
        gy += wgt * (yr * rr + yi * ri);
        gz += wgt * (zr * rr + zi * ri);
    }
}

// Potential and gradient: one thread per body (sorted order), so that every lane has work
// whatever the leaf sizes (a leaf holds at most ncrit bodies, often far fewer than a
// wave).  Each thread reads its leaf's coefficients at compile-time offsets from its own
// base; the lanes of one leaf read the same addresses.
template <int P>
__global__ void __launch_bounds__(256) k_l2p(const int32_t *body_leaf, int64_t n, Geo g, const float4 *bodies,
                                             const float *L, float4 *out) {
    using D = Dims<P>;
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= n) return;
    const int c = body_leaf[b];
    double cx, cy, cz, inv;
    cell_center(g.level[c], g.ix[c], g.iy[c], g.iz[c], g.x0x, g.x0y, g.x0z, g.k, cx, cy, cz, inv);
    const float finv = (float)inv;
    const float *v = L + (int64_t)c * D::KP;
    const float4 bd = bodies[b];
    const float ux = (float)(((double)bd.x - cx) * inv);
    const float uy = (float)(((double)bd.y - cy) * inv);
    const float uz = (float)(((double)bd.z - cz) * inv);
    float f = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
    stream_regular<P>(ux, uy, uz,
                      [&](int l, int m, float rr, float ri) { l2p_term<P>(v, l, m, rr, ri, f, gx, gy, gz); });
    const float g2 = finv * finv;
    out[b] = make_float4(f * finv, gx * g2, gy * g2, gz * g2);   // potential, gradient
}

// Potential, gradient and Hessian: one wave per leaf, the local coefficients broadcast
// from LDS.  The harmonic stream stays rolled and the coefficients are indexed at run time
// (unrolled, the six Hessian expansions keep too many values live: one wave per SIMD and a
// register spill at p >= 9).  The gradient of a local expansion is again a local
// expansion (the map in l2p_term), so the six Hessian expansions (degree <= p-2) are built
// once per leaf in LDS by applying that map twice.
template <int P>
__global__ void __launch_bounds__(64) k_l2p_hess(const int32_t *leaves, Geo g, const float4 *bodies, const float *L,
                                                 float4 *out, float *out_h) {
    using D = Dims<P>;
    constexpr int KP = D::KP;
    constexpr int NT1 = P >= 1 ? P * (P + 1) / 2 : 1;          // (l, m >= 0) pairs with l <= P-1
    constexpr int NT2 = P >= 2 ? (P - 1) * P / 2 : 1;          // l <= P-2
    __shared__ float sL[KP];
    __shared__ float cre[3][NT1], cim[3][NT1];
    __shared__ float hre[6][NT2], him[6][NT2];
    const int c = leaves[blockIdx.x];
    const int lane = threadIdx.x;
    for (int d = lane; d < KP; d += 64) sL[d] = L[(int64_t)c * KP + d];
    __syncthreads();
    const int s = g.start[c], n = g.count[c];
    double cx, cy, cz, inv;
    cell_center(g.level[c], g.ix[c], g.iy[c], g.iz[c], g.x0x, g.x0y, g.x0z, g.k, cx, cy, cz, inv);
    const float finv = (float)inv;
    const float *vL = sL;
    auto lre = [&](int j, int m) { return loc_re(vL, j, m); };
    auto lim = [&](int j, int m) { return loc_im(vL, j, m); };
    if (P >= 2) {
        // gradient expansions C^a, degree <= P-1
        for (int e = lane; e < NT1; e += 64) {
            int l = 0;
            while ((l + 1) * (l + 2) / 2 <= e) ++l;
            const int m = e - l * (l + 1) / 2;
            const float zr = lre(l + 1, m), zi = lim(l + 1, m);
            const float pr = lre(l + 1, m + 1), pi = lim(l + 1, m + 1);
            const float mr = lre(l + 1, m - 1), mi = lim(l + 1, m - 1);
            cre[0][e] = 0.5f * (mr - pr); cim[0][e] = 0.5f * (mi - pi);
            cre[1][e] = -0.5f * (pi + mi); cim[1][e] = 0.5f * (pr + mr);
            cre[2][e] = zr; cim[2][e] = zi;
        }
        __syncthreads();
        // Hessian expansions H^{ab} = d_b C^a, degree <= P-2, order xx yy zz xy xz yz
        for (int e = lane; e < 6 * NT2; e += 64) {
            const int comp = e / NT2, t = e % NT2;
            int l = 0;
            while ((l + 1) * (l + 2) / 2 <= t) ++l;
            const int m = t - l * (l + 1) / 2;
            const int A = comp < 3 ? comp : (comp < 5 ? 0 : 1);
            const int B = comp < 3 ? comp : (comp == 3 ? 1 : 2);
            auto cr = [&](int j, int mm) -> float {
                if (mm > j) return 0.f;
                if (mm >= 0) return cre[A][j * (j + 1) / 2 + mm];
                return -cre[A][j * (j + 1) / 2 + 1];           // C_{j,-1} = -conj(C_{j,1})
            };
            auto ci = [&](int j, int mm) -> float {
                if (mm > j) return 0.f;
                if (mm >= 0) return cim[A][j * (j + 1) / 2 + mm];
                return cim[A][j * (j + 1) / 2 + 1];
            };
            const float zr = cr(l + 1, m), zi = ci(l + 1, m);
            const float pr = cr(l + 1, m + 1), pi = ci(l + 1, m + 1);
            const float mr = cr(l + 1, m - 1), mi = ci(l + 1, m - 1);
            float hr, hi;
            if (B == 0) { hr = 0.5f * (mr - pr); hi = 0.5f * (mi - pi); }
            else if (B == 1) { hr = -0.5f * (pi + mi); hi = 0.5f * (pr + mr); }
            else { hr = zr; hi = zi; }
            hre[comp][t] = hr;
            him[comp][t] = hi;
        }
        __syncthreads();
    }
    for (int base = 0; base < n; base += 64) {
        const int j = base + lane;
        if (j >= n) break;
        float4 b = bodies[s + j];
        const float ux = (float)(((double)b.x - cx) * inv);
        const float uy = (float)(((double)b.y - cy) * inv);
        const float uz = (float)(((double)b.z - cz) * inv);
        float f = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
        float h[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        auto term = [&](int l, int m, float rr, float ri) {
            l2p_term<P>(vL, l, m, rr, ri, f, gx, gy, gz);
            const float wgt = m == 0 ? 1.f : 2.f;
            if (l + 2 <= P) {
                const int t = l * (l + 1) / 2 + m;
                h[0] += wgt * (hre[0][t] * rr + him[0][t] * ri);
                h[1] += wgt * (hre[1][t] * rr + him[1][t] * ri);
                h[2] += wgt * (hre[2][t] * rr + him[2][t] * ri);
                h[3] += wgt * (hre[3][t] * rr + him[3][t] * ri);
                h[4] += wgt * (hre[4][t] * rr + him[4][t] * ri);
                h[5] += wgt * (hre[5][t] * rr + him[5][t] * ri);
            }
        };
        stream_regular_rolled<P>(ux, uy, uz, term);
        const float g2 = finv * finv;
        out[s + j] = make_float4(f * finv, gx * g2, gy * g2, gz * g2);   // potential, gradient
        const float g3 = g2 * finv;
#pragma unroll
        for (int q = 0; q < 6; ++q) out_h[(int64_t)(s + j) * 6 + q] = h[q] * g3;
    }
}

// ------------------------------------------------------------------ P2P
constexpr int kP2PBatch = 1024;

// One target against sources src[g], src[g + G], ... (charges in .w); with DIP the
// sources also carry dipoles (srcd[j].xyz): a dipole g at x_j adds g.d / r^3 to the
// potential and g / r^3 - 3 (g.d) d / r^5 to its gradient (d = x_i - x_j).
template <bool CHECK, bool DIP = false>
__device__ __forceinline__ void p2p_batch(const float4 *src, const float4 *srcd, int ns, int g, int G, float xi,
                                          float yi, float zi, float &f, float &gx, float &gy, float &gz) {
    int jj = g;
#pragma unroll 4
    for (; jj < ns; jj += G) {
        const float4 sj = src[jj];
        const float dx = xi - sj.x, dy = yi - sj.y, dz = zi - sj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        float inv = __builtin_amdgcn_rsqf(r2);
        if (CHECK) inv = r2 > 0.f ? inv : 0.f;
        const float qi = sj.w * inv;
        const float qi3 = qi * inv * inv;
        f += qi;
        gx -= dx * qi3;
        gy -= dy * qi3;
        gz -= dz * qi3;
        if (DIP) {
            const float4 dj = srcd[jj];
            const float inv3 = inv * inv * inv;
            const float t = (dj.x * dx + dj.y * dy + dj.z * dz) * inv3;
            const float t5 = 3.f * t * inv * inv;
            f += t;
            gx += dj.x * inv3 - t5 * dx;
            gy += dj.y * inv3 - t5 * dy;
            gz += dj.z * inv3 - t5 * dz;
        }
    }
}

// Compensated accumulation: sums over blocks of 16 sources are added to (hi, lo) pairs
// with Knuth's TwoSum, so the rounding error of the running sum is carried in lo.
struct Comp4 {
    float h[4] = {0.f, 0.f, 0.f, 0.f}, l[4] = {0.f, 0.f, 0.f, 0.f};
    __device__ __forceinline__ void add(int i, float b) {
        const float s = h[i] + b;
        const float bb = s - h[i];
        const float err = (h[i] - (s - bb)) + (b - bb);
        h[i] = s;
        l[i] += err;
    }
};

template <bool CHECK, bool DIP = false>
__device__ __forceinline__ void p2p_batch_comp(const float4 *src, const float4 *srcd, int ns, int g, int G, float xi,
                                               float yi, float zi, Comp4 &c) {
    for (int j0 = g; j0 < ns; j0 += 16 * G) {
        float f = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
        const int j1 = min(ns, j0 + 16 * G);
        p2p_batch<CHECK, DIP>(src + j0 - g, DIP ? srcd + j0 - g : srcd, j1 - (j0 - g), g, G, xi, yi, zi, f, gx, gy, gz);
        c.add(0, f);
        c.add(1, gx);
        c.add(2, gy);
        c.add(3, gz);
    }
}

// Source runs of a target leaf, streamed through the LDS batch `src`: the run descriptors
// are read kP2PThreads at a time (one per thread) and their lengths scanned, so that the
// bodies of many short runs are copied in one parallel pass (an adaptive tree can give a
// coarse leaf tens of thousands of small source leaves).  Only the sources whose position
// in the leaf's concatenated source list lies in [lo, hi) are taken (run_pre: exclusive
// prefix of all run lengths, base = its value at the leaf's first run).  flush(n)
// consumes the n staged sources; it is called when the batch is full and at the end.
// With `dips`, the sources' dipoles are staged in `srcd` beside them.  Every thread of the
// block calls this with the same arguments.
struct RunStage {
    int st[kP2PThreads];        // first body of each run of the chunk
    int off[kP2PThreads + 1];   // exclusive prefix of the run lengths
    int wsum[kP2PThreads / 64];
};
template <class Flush>
__device__ __forceinline__ void p2p_stream_runs(const int2 *segs, const int64_t *run_pre, int sg0, int sg1, int64_t base,
                                                int64_t lo, int64_t hi, const float4 *bodies, float4 *src,
                                                RunStage &rs, Flush flush, const float4 *dips = nullptr,
                                                float4 *srcd = nullptr) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int pos = 0;
    for (int c0 = sg0; c0 < sg1; c0 += kP2PThreads) {
        const int nr = min(kP2PThreads, sg1 - c0);
        int st = 0, len = 0;
        if (tid < nr) {
            const int2 r = segs[c0 + tid];
            const int64_t pre = run_pre[c0 + tid] - base, a = max(pre, lo), b = min(pre + r.y, hi);
            st = r.x + (int)(a - pre);
            len = b > a ? (int)(b - a) : 0;
        }
        int incl = len;   // block-wide inclusive scan of the lengths
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) rs.wsum[wave] = incl;
        __syncthreads();
        for (int w = 0; w < wave; ++w) incl += rs.wsum[w];
        rs.st[tid] = st;
        rs.off[tid + 1] = incl;
        if (tid == 0) rs.off[0] = 0;
        __syncthreads();
        const int total = rs.off[nr];
        for (int b0 = 0; b0 < total;) {
            const int take = min(total - b0, kP2PBatch - pos);
            if (pos == 0) __syncthreads();   // the previous batch has been consumed
            for (int i = tid; i < take; i += kP2PThreads) {
                const int e = b0 + i;
                int l = 0, h = nr - 1;       // the run holding element e: last r with off[r] <= e
                while (l < h) {
                    const int mid = (l + h + 1) >> 1;
                    if (rs.off[mid] <= e) l = mid;
                    else h = mid - 1;
                }
                src[pos + i] = bodies[rs.st[l] + (e - rs.off[l])];
                if (dips) srcd[pos + i] = dips[rs.st[l] + (e - rs.off[l])];
            }
            pos += take;
            b0 += take;
            if (pos == kP2PBatch) {
                __syncthreads();
                flush(pos);
                pos = 0;
            }
        }
        __syncthreads();   // rs is rewritten by the next chunk
    }
    if (pos > 0) {
        __syncthreads();
        flush(pos);
    }
}

// A near-field work item (leaf, piece j of k, first partial block): a leaf whose list
// holds more than kP2PPieceWork interactions is cut into k pieces of about equal source
// counts, each written as a partial result and summed by k_p2p_join in piece order
// (deterministic); k = 1 leaves write their result directly.  The run range of piece j:
struct P2PPiece {
    int sg0, sg1;          // runs that overlap the piece
    int64_t base, lo, hi;  // run_pre at the leaf's first run, and the piece's source range
};
__device__ inline P2PPiece p2p_piece(const int32_t *seg_off, const int64_t *run_pre, int li, int j, int k) {
    P2PPiece pc;
    pc.sg0 = seg_off[li];
    pc.sg1 = seg_off[li + 1];
    pc.base = run_pre[pc.sg0];
    const int64_t S = run_pre[pc.sg1] - pc.base;
    pc.lo = S * j / k;
    pc.hi = S * (j + 1) / k;
    if (k > 1) {   // the first run ending after lo, the first run starting at or after hi
        int l = pc.sg0, h = pc.sg1;
        while (l < h) {
            const int m = (l + h) >> 1;
            if (run_pre[m + 1] - pc.base <= pc.lo) l = m + 1;
            else h = m;
        }
        const int a = l;
        l = a;
        h = pc.sg1;
        while (l < h) {
            const int m = (l + h) >> 1;
            if (run_pre[m] - pc.base < pc.hi) l = m + 1;
            else h = m;
        }
        pc.sg0 = a;
        pc.sg1 = l;
    }
    return pc;
}

template <bool COMP, bool DIP = false>
__global__ void __launch_bounds__(kP2PThreads) k_p2p(const int4 *items, const int32_t *leaves, const int32_t *c_start,
                                                     const int32_t *c_count, const int32_t *seg_off, const int2 *segs,
                                                     const int64_t *run_pre, const float4 *bodies, float4 *out,
                                                     float4 *part, const float4 *dips = nullptr) {
    __shared__ float4 src[kP2PBatch];
    __shared__ float4 srcd[DIP ? kP2PBatch : 1];
    __shared__ float4 red[kP2PThreads];
    __shared__ float4 redl[COMP ? kP2PThreads : 1];
    __shared__ RunStage rs;
    const int4 item = items[blockIdx.x];
    const int li = item.x, piece = item.y, npieces = item.z;
    const int c = leaves[li];
    const int ts = c_start[c], tn = c_count[c];
    const int tid = threadIdx.x;
    const P2PPiece pc = p2p_piece(seg_off, run_pre, li, piece, npieces);
    for (int t0 = 0; t0 < tn; t0 += kP2PThreads) {
        const int nt = min(kP2PThreads, tn - t0);
        const int G = kP2PThreads / nt;
        const bool active = tid < nt * G;
        const int t = tid % nt, g = tid / nt;
        float xi = 0.f, yi = 0.f, zi = 0.f;
        if (active) {
            float4 b = bodies[ts + t0 + t];
            xi = b.x; yi = b.y; zi = b.z;
        }
        float f = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
        Comp4 cmp;
        // the target leaf itself (first piece): skip j == i and coincident points
        for (int s0 = 0; piece == 0 && s0 < tn; s0 += kP2PBatch) {
            const int ns = min(kP2PBatch, tn - s0);
            __syncthreads();
            for (int i = tid; i < ns; i += kP2PThreads) {
                src[i] = bodies[ts + s0 + i];
                if (DIP) srcd[i] = dips[ts + s0 + i];
            }
            __syncthreads();
            if (active) {
                if (COMP) p2p_batch_comp<true, DIP>(src, srcd, ns, g, G, xi, yi, zi, cmp);
                else p2p_batch<true, DIP>(src, srcd, ns, g, G, xi, yi, zi, f, gx, gy, gz);
            }
        }
        // neighbouring leaves, batched through LDS
        p2p_stream_runs(
            segs, run_pre, pc.sg0, pc.sg1, pc.base, pc.lo, pc.hi, bodies, src, rs,
            [&](int ns) {
                if (active) {
                    if (COMP) p2p_batch_comp<false, DIP>(src, srcd, ns, g, G, xi, yi, zi, cmp);
                    else p2p_batch<false, DIP>(src, srcd, ns, g, G, xi, yi, zi, f, gx, gy, gz);
                }
            },
            DIP ? dips : nullptr, DIP ? srcd : nullptr);
        __syncthreads();
        if (COMP) {
            red[tid] = make_float4(cmp.h[0], cmp.h[1], cmp.h[2], cmp.h[3]);
            redl[tid] = make_float4(cmp.l[0], cmp.l[1], cmp.l[2], cmp.l[3]);
        } else {
            red[tid] = make_float4(f, gx, gy, gz);
        }
        __syncthreads();
        if (tid < nt) {
            float4 acc = red[tid];
            if (COMP) {
                Comp4 tot;
                float lsum[4] = {0.f, 0.f, 0.f, 0.f};
                for (int gg = 0; gg < G; ++gg) {
                    const float4 v = red[gg * nt + tid], vl = redl[gg * nt + tid];
                    tot.add(0, v.x); tot.add(1, v.y); tot.add(2, v.z); tot.add(3, v.w);
                    lsum[0] += vl.x; lsum[1] += vl.y; lsum[2] += vl.z; lsum[3] += vl.w;
                }
                acc = make_float4(tot.h[0] + (tot.l[0] + lsum[0]), tot.h[1] + (tot.l[1] + lsum[1]),
                                  tot.h[2] + (tot.l[2] + lsum[2]), tot.h[3] + (tot.l[3] + lsum[3]));
            } else {
                for (int gg = 1; gg < G; ++gg) {
                    float4 v = red[gg * nt + tid];
                    acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
                }
            }
            if (npieces == 1) out[ts + t0 + tid] = acc;   // potential, gradient
            else part[(int64_t)(item.w + piece) * kP2PThreads + tid] = acc;   // split leaves have tn <= kP2PThreads
        }
    }
}

// Sum of the pieces of every split leaf, in piece order.
__global__ void __launch_bounds__(kP2PThreads) k_p2p_join(const int4 *items, const int32_t *leaves,
                                                          const int32_t *c_start, const int32_t *c_count,
                                                          const float4 *part, float4 *out, const float *part_h,
                                                          float *out_h) {
    const int4 item = items[blockIdx.x];
    if (item.y != 0 || item.z == 1) return;
    const int c = leaves[item.x];
    const int ts = c_start[c], tn = c_count[c], t = threadIdx.x;
    if (t >= tn) return;
    Comp4 acc;   // compensated, so that splitting keeps the mixed-precision near field's accuracy
    float h[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < item.z; ++j) {
        const int64_t b = (int64_t)(item.w + j) * kP2PThreads + t;
        const float4 v = part[b];
        acc.add(0, v.x); acc.add(1, v.y); acc.add(2, v.z); acc.add(3, v.w);
        if (out_h)
            for (int q = 0; q < 6; ++q) h[q] += part_h[b * 6 + q];
    }
    out[ts + t] = make_float4(acc.h[0] + acc.l[0], acc.h[1] + acc.l[1], acc.h[2] + acc.l[2], acc.h[3] + acc.l[3]);
    if (out_h)
        for (int q = 0; q < 6; ++q) out_h[(int64_t)(ts + t) * 6 + q] = h[q];
}

// Near field with the Hessian of the potential as well (losses through grad phi):
// per interaction H += q (3 d d^T / r^5 - I / r^3), d = x_i - x_j.  Same layout and
// batching as k_p2p; FP32 accumulation.
template <bool CHECK>
__device__ __forceinline__ void p2p_batch_h(const float4 *src, int ns, int g, int G, float xi, float yi, float zi,
                                            float *a) {
    for (int jj = g; jj < ns; jj += G) {
        const float4 sj = src[jj];
        const float dx = xi - sj.x, dy = yi - sj.y, dz = zi - sj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        float inv = __builtin_amdgcn_rsqf(r2);
        if (CHECK) inv = r2 > 0.f ? inv : 0.f;
        const float inv2 = inv * inv;
        const float qi = sj.w * inv, qi3 = qi * inv2, qi5 = 3.f * qi3 * inv2;
        a[0] += qi;
        a[1] -= dx * qi3; a[2] -= dy * qi3; a[3] -= dz * qi3;
        a[4] += qi5 * dx * dx - qi3; a[5] += qi5 * dy * dy - qi3; a[6] += qi5 * dz * dz - qi3;
        a[7] += qi5 * dx * dy; a[8] += qi5 * dx * dz; a[9] += qi5 * dy * dz;
    }
}

__global__ void __launch_bounds__(kP2PThreads) k_p2p_hess(const int4 *items, const int32_t *leaves,
                                                          const int32_t *c_start, const int32_t *c_count,
                                                          const int32_t *seg_off, const int2 *segs,
                                                          const int64_t *run_pre, const float4 *bodies, float4 *out,
                                                          float *out_h, float4 *part, float *part_h) {
    __shared__ float4 src[kP2PBatch];
    __shared__ float red[10][kP2PThreads];
    __shared__ RunStage rs;
    const int4 item = items[blockIdx.x];
    const int li = item.x, piece = item.y, npieces = item.z;
    const int c = leaves[li];
    const int ts = c_start[c], tn = c_count[c];
    const int tid = threadIdx.x;
    const P2PPiece pc = p2p_piece(seg_off, run_pre, li, piece, npieces);
    for (int t0 = 0; t0 < tn; t0 += kP2PThreads) {
        const int nt = min(kP2PThreads, tn - t0);
        const int G = kP2PThreads / nt;
        const bool active = tid < nt * G;
        const int t = tid % nt, g = tid / nt;
        float xi = 0.f, yi = 0.f, zi = 0.f;
        if (active) {
            float4 b = bodies[ts + t0 + t];
            xi = b.x; yi = b.y; zi = b.z;
        }
        float a[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int s0 = 0; piece == 0 && s0 < tn; s0 += kP2PBatch) {     // the target leaf itself
            const int ns = min(kP2PBatch, tn - s0);
            __syncthreads();
            for (int i = tid; i < ns; i += kP2PThreads) src[i] = bodies[ts + s0 + i];
            __syncthreads();
            if (active) p2p_batch_h<true>(src, ns, g, G, xi, yi, zi, a);
        }
        p2p_stream_runs(segs, run_pre, pc.sg0, pc.sg1, pc.base, pc.lo, pc.hi, bodies, src, rs, [&](int ns) {
            if (active) p2p_batch_h<false>(src, ns, g, G, xi, yi, zi, a);
        });
        __syncthreads();
        for (int q = 0; q < 10; ++q) red[q][tid] = a[q];
        __syncthreads();
        if (tid < nt) {
            float acc[10];
            for (int q = 0; q < 10; ++q) {
                acc[q] = red[q][tid];
                for (int gg = 1; gg < G; ++gg) acc[q] += red[q][gg * nt + tid];
            }
            const float4 v = make_float4(acc[0], acc[1], acc[2], acc[3]);
            if (npieces == 1) {
                out[ts + t0 + tid] = v;
                for (int q = 0; q < 6; ++q) out_h[(int64_t)(ts + t0 + tid) * 6 + q] = acc[4 + q];
            } else {
                const int64_t b = (int64_t)(item.w + piece) * kP2PThreads + tid;
                part[b] = v;
                for (int q = 0; q < 6; ++q) part_h[b * 6 + q] = acc[4 + q];
            }
        }
    }
}

// ------------------------------------------------------------------ permutes
__global__ void k_set_charges(const float *q, const int32_t *perm, int64_t n, float4 *bodies) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bodies[i].w = q[perm[i]];
}

// Dipoles ([n][3], input order) into sorted order.
__global__ void k_set_dipoles(const float *g, const int32_t *perm, int64_t n, float4 *dip) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = perm[i];
        dip[i] = make_float4(g[3 * o], g[3 * o + 1], g[3 * o + 2], 0.f);
    }
}
// The bodies with component a of their dipole as charge.
__global__ void k_bodies_component(const float4 *bodies, const float4 *dip, int a, int64_t n, float4 *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 b = bodies[i], d = dip[i];
        out[i] = make_float4(b.x, b.y, b.z, a == 0 ? d.x : (a == 1 ? d.y : d.z));
    }
}

// Multipoles of dipole sources.  A dipole g at x is the derivative of a unit charge's
// multipole conj(R_lm(u)) (u = (x - c) / side) as the charge moves along g, and the
// derivatives of the regular harmonics are harmonics of one degree less:
//   d_x R_lm = (R_{l-1,m+1} - R_{l-1,m-1}) / 2,  d_y R_lm = -i (R_{l-1,m-1} + R_{l-1,m+1}) / 2,
//   d_z R_lm = R_{l-1,m},  with R_{l,-1} = -conj(R_{l,1}).
// So with M^a the multipoles of the charges g_a (a = x, y, z, made by k_p2m), the dipoles
// add to M_lm, per leaf, (1/side) [M^z_{l-1,m} + (M^x_{l-1,m+1} - M^x_{l-1,m-1}) / 2
//   + i (M^y_{l-1,m-1} + M^y_{l-1,m+1}) / 2].
template <int P>
__global__ void k_dip_combine(const int32_t *leaves, int64_t nleaves, Geo g, const float *Mdip, int64_t ncells,
                              float *M) {
    using D = Dims<P>;
    constexpr int KP = D::KP, NT = (P + 1) * (P + 2) / 2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nleaves * NT;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = leaves[i / NT];
        const int t = (int)(i % NT);
        int l = 0;
        while ((l + 1) * (l + 2) / 2 <= t) ++l;
        const int m = t - l * (l + 1) / 2;
        if (l == 0) continue;
        // coefficient (j, mm) of the multipole of component a, mm >= -1
        auto get = [&](int a, int j, int mm, float &re, float &im) {
            const float *Ma = Mdip + ((int64_t)a * ncells + c) * KP;
            re = im = 0.f;
            if (mm > j || -mm > j) return;
            if (mm == 0) { re = Ma[j * j]; return; }
            if (mm > 0) { re = Ma[j * j + 2 * mm - 1]; im = Ma[j * j + 2 * mm]; return; }
            re = -Ma[j * j + 1];                // M_{j,-1} = -conj(M_{j,1})
            im = Ma[j * j + 2];
        };
        float zr, zi, xpr, xpi, xmr, xmi, ypr, ypi, ymr, ymi;
        get(2, l - 1, m, zr, zi);
        get(0, l - 1, m + 1, xpr, xpi);
        get(0, l - 1, m - 1, xmr, xmi);
        get(1, l - 1, m + 1, ypr, ypi);
        get(1, l - 1, m - 1, ymr, ymi);
        const float dr = zr + 0.5f * (xpr - xmr) - 0.5f * (ymi + ypi);
        const float di = zi + 0.5f * (xpi - xmi) + 0.5f * (ymr + ypr);
        double cx, cy, cz, inv;
        cell_center(g.level[c], g.ix[c], g.iy[c], g.iz[c], g.x0x, g.x0y, g.x0z, g.k, cx, cy, cz, inv);
        const float fi = (float)inv;
        float *Mc = M + (int64_t)c * KP;
        if (m == 0) {
            Mc[l * l] += fi * dr;
        } else {
            Mc[l * l + 2 * m - 1] += fi * dr;
            Mc[l * l + 2 * m] += fi * di;
        }
    }
}

// Far + near field back to input order: one thread per output (coalesced writes), the
// sorted-order inputs are gathered through the inverse permutation.
__global__ void k_combine(const int32_t *iperm, int64_t n, const float4 *far, const float4 *near, float *phi,
                          float *grad) {
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = iperm[o];
        const float4 f = far[i], c = near[i];
        if (phi) phi[o] = f.x + c.x;
        if (grad) {
            grad[3 * o] = f.y + c.y;
            grad[3 * o + 1] = f.z + c.z;
            grad[3 * o + 2] = f.w + c.w;
        }
    }
}

__global__ void k_combine_hess(const int32_t *iperm, int64_t n, const float *farh, const float *nearh, float *hess) {
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = iperm[o];
#pragma unroll
        for (int q = 0; q < 6; ++q) hess[6 * o + q] = farh[6 * i + q] + nearh[6 * i + q];
    }
}

// dL/dx_i = w_i grad phi_i + q_i grad psi_i (input order)
__global__ void k_adjoint_combine(int64_t n, const float *w, const float *gphi, const float *q, const float *gpsi,
                                  float *dx) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float wi = w[i], qi = q[i];
        dx[3 * i] = wi * gphi[3 * i] + qi * gpsi[3 * i];
        dx[3 * i + 1] = wi * gphi[3 * i + 1] + qi * gpsi[3 * i + 1];
        dx[3 * i + 2] = wi * gphi[3 * i + 2] + qi * gpsi[3 * i + 2];
    }
}

// dL/dx = w E + H g + q grad Psi (input order; H as xx yy zz xy xz yz; see run_adjoint_grad)
__global__ void k_adjoint_dip_final(int64_t n, const float *w, const float *E, const float *q, const float *gpsi,
                                    const float *H, const float *g, float *dx) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float *h = H + 6 * i;
        const float gx = g[3 * i], gy = g[3 * i + 1], gz = g[3 * i + 2];
        const float hg[3] = {h[0] * gx + h[3] * gy + h[4] * gz, h[3] * gx + h[1] * gy + h[5] * gz,
                             h[4] * gx + h[5] * gy + h[2] * gz};
        for (int r = 0; r < 3; ++r) dx[3 * i + r] = w[i] * E[3 * i + r] + hg[r] + q[i] * gpsi[3 * i + r];
    }
}

// ------------------------------------------------------------------ host side
static int grid1(int64_t n, int bs = 256) {
    int64_t g = (n + bs - 1) / bs;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}

enum { PH_PERM = 0, PH_P2M, PH_M2M, PH_M2L, PH_L2L, PH_L2P, PH_P2P, PH_COMB, PH_TOTAL };

static inline void ev_rec(fmm_plan_s *Pl, int slot, hipStream_t s) {
    if (Pl->timing) HIP_CHECK(hipEventRecord(Pl->ev[slot], s));
}

// Near field on the side stream, forked from the main stream at the point where this is
// called; the main stream joins it (ev_join) before the outputs are combined.
static void launch_near(fmm_plan_s *Pl, int phases, bool hess, hipStream_t s) {
    HIP_CHECK(hipEventRecord(Pl->ev_fork, s));
    HIP_CHECK(hipStreamWaitEvent(Pl->side, Pl->ev_fork, 0));
    ev_rec(Pl, 2 * PH_P2P, Pl->side);
    if ((phases & FMM_NEAR) && hess) {
        hipLaunchKernelGGL(k_p2p_hess, (int)Pl->np2p_items, kP2PThreads, 0, Pl->side, (const int4 *)Pl->p2p_items,
                           (const int32_t *)Pl->leaves, (const int32_t *)Pl->c_start, (const int32_t *)Pl->c_count,
                           (const int32_t *)Pl->seg_off, (const int2 *)Pl->segs, (const int64_t *)Pl->run_pre,
                           (const float4 *)Pl->bodies, Pl->near4, Pl->nearh, Pl->p2p_part, Pl->p2p_part_h);
        if (Pl->np2p_part > 0)
            hipLaunchKernelGGL(k_p2p_join, (int)Pl->np2p_items, kP2PThreads, 0, Pl->side, (const int4 *)Pl->p2p_items,
                               (const int32_t *)Pl->leaves, (const int32_t *)Pl->c_start, (const int32_t *)Pl->c_count,
                               (const float4 *)Pl->p2p_part, Pl->near4, (const float *)Pl->p2p_part_h, Pl->nearh);
    } else if (phases & FMM_NEAR) {
        const bool comp = Pl->prec == FMM_PREC_MIXED;
        auto kern = Pl->dip_on ? (comp ? k_p2p<true, true> : k_p2p<false, true>)
                               : (comp ? k_p2p<true, false> : k_p2p<false, false>);
        hipLaunchKernelGGL(kern, (int)Pl->np2p_items, kP2PThreads, 0, Pl->side, (const int4 *)Pl->p2p_items,
                           (const int32_t *)Pl->leaves, (const int32_t *)Pl->c_start, (const int32_t *)Pl->c_count,
                           (const int32_t *)Pl->seg_off, (const int2 *)Pl->segs, (const int64_t *)Pl->run_pre,
                           (const float4 *)Pl->bodies, Pl->near4, Pl->p2p_part,
                           (const float4 *)(Pl->dip_on ? Pl->dip : nullptr));
        if (Pl->np2p_part > 0)
            hipLaunchKernelGGL(k_p2p_join, (int)Pl->np2p_items, kP2PThreads, 0, Pl->side, (const int4 *)Pl->p2p_items,
                               (const int32_t *)Pl->leaves, (const int32_t *)Pl->c_start, (const int32_t *)Pl->c_count,
                               (const float4 *)Pl->p2p_part, Pl->near4, (const float *)nullptr, (float *)nullptr);
    } else {
        fill_f32(reinterpret_cast<float *>(Pl->near4), 0.f, 4 * Pl->n, Pl->side);
        if (hess) fill_f32(Pl->nearh, 0.f, 6 * Pl->n, Pl->side);
    }
    ev_rec(Pl, 2 * PH_P2P + 1, Pl->side);
    HIP_CHECK(hipEventRecord(Pl->ev_join, Pl->side));
}

// The near field (near(), on the side stream) is forked before P2M and runs beside P2M and
// the M2M levels.  Forking it right before M2L instead frees those small launches but
// slows M2L by nearly the P2P time (at p = 12 a near-field workgroup fits beside two M2L
// workgroups on a compute unit, yet 17.6 ms of P2P still added 14.4 ms to M2L).
template <int P, class Near> static void far_field(fmm_plan_s *Pl, const Geo &g, hipStream_t s, const Near &near) {
    using D = Dims<P>;
    const OpTables &T = op_tables(P);
    const bool mixed = Pl->prec == FMM_PREC_MIXED;
    const int RL = mixed ? kRootLevels : 0;       // levels below RL accumulate in FP64
    constexpr unsigned kSlabs = (D::KP + kSlab64 - 1) / kSlab64;
    near();
    ev_rec(Pl, 2 * PH_P2M, s);
    hipLaunchKernelGGL(k_p2m<P>, (int)((Pl->nleaves + 1) / 2), 64, 0, s, (const int32_t *)Pl->leaves, Pl->nleaves,
                       g, (const float4 *)Pl->bodies, Pl->M);
    if (Pl->dip_on) {
        // dipole sources: leaf multipoles of each dipole component as charges, then the
        // degree-raising combination into M
        for (int a = 0; a < 3; ++a) {
            hipLaunchKernelGGL(k_bodies_component, grid1(Pl->n), 256, 0, s, (const float4 *)Pl->bodies,
                               (const float4 *)Pl->dip, a, Pl->n, Pl->dipb);
            hipLaunchKernelGGL(k_p2m<P>, (int)((Pl->nleaves + 1) / 2), 64, 0, s, (const int32_t *)Pl->leaves,
                               Pl->nleaves, g, (const float4 *)Pl->dipb, Pl->Mdip + (int64_t)a * Pl->ncells * D::KP);
        }
        hipLaunchKernelGGL(k_dip_combine<P>, grid1(Pl->nleaves * (int64_t)((P + 1) * (P + 2) / 2)), 256, 0, s,
                           (const int32_t *)Pl->leaves, Pl->nleaves, g, (const float *)Pl->Mdip, Pl->ncells, Pl->M);
    }
    ev_rec(Pl, 2 * PH_P2M + 1, s);
    ev_rec(Pl, 2 * PH_M2M, s);
    for (int l = Pl->max_level - 1; l >= RL; --l) {
        const int t0 = Pl->m2m.bucket_tile[l * 8], t1 = Pl->m2m.bucket_tile[l * 8 + 8];
        if (t1 > t0)
            hipLaunchKernelGGL((k_gemm<P, false, false>), t1 - t0, 256, 0, s, (const int4 *)Pl->m2m.work + t0,
                               (const int32_t *)Pl->m2m.entry_key, (const int32_t *)Pl->m2m.entry_src,
                               (const uint8_t *)nullptr, T.m2m_ptrs, (const float *)Pl->M, Pl->M, (float *)nullptr,
                               (const int32_t *)Pl->m2m.tile_targets);
    }
    if (mixed) {
        hipLaunchKernelGGL(k_root_leaves_to64, grid1(Pl->nroot * D::KP), 256, 0, s, Pl->nroot, D::KP,
                           (const int32_t *)Pl->c_nchild, (const float *)Pl->M, Pl->Md);
        for (int l = std::min(RL - 1, Pl->max_level - 1); l >= 0; --l) {
            const int t0 = Pl->m2m.bucket_tile[l * 8], t1 = Pl->m2m.bucket_tile[l * 8 + 8];
            if (t1 > t0)
                hipLaunchKernelGGL((k_gemm64<P, false>), dim3(t1 - t0, kSlabs), 256, 0, s, (const int4 *)Pl->m2m.work + t0,
                                   (const int32_t *)Pl->m2m.entry_key, (const int32_t *)Pl->m2m.entry_src,
                                   T.m2m64_ptrs, Pl->nroot, (const float *)Pl->M, (const double *)Pl->Md, Pl->Md,
                                   (double *)nullptr, (const int32_t *)Pl->m2m.tile_targets);
        }
        hipLaunchKernelGGL(k_root_to32, grid1(Pl->nroot * D::KP), 256, 0, s, Pl->nroot, D::KP,
                           (const double *)Pl->Md, Pl->M);
        hipLaunchKernelGGL(k_split_m<P>, (int)Pl->ncells, 64, 0, s, (const float *)Pl->M, T.nu, Pl->Mh, Pl->Ml,
                           Pl->Msinv);
    }
    ev_rec(Pl, 2 * PH_M2M + 1, s);
    fill_f32(Pl->L, 0.f, Pl->ncells * (int64_t)D::KP, s);
    if (mixed) fill_f32(reinterpret_cast<float *>(Pl->Ld), 0.f, 2 * Pl->nroot * (int64_t)D::KP, s);
    ev_rec(Pl, 2 * PH_M2L, s);
    // mixed precision: the FP64 root-level M2L is a small launch that writes only Ld (and
    // its partials), so it runs on the side stream (after the near field queued there)
    // beside the main M2L launch; the main stream waits for it before reading Ld.  ev_join
    // recorded after it still covers the near field before it.
    const bool root_side = mixed && Pl->nwork64 > 0;
    if (root_side) {
        HIP_CHECK(hipEventRecord(Pl->ev_fork, s));
        HIP_CHECK(hipStreamWaitEvent(Pl->side, Pl->ev_fork, 0));
        hipLaunchKernelGGL((k_gemm64<P, false>), dim3((unsigned)Pl->nwork64, kSlabs), 256, 0, Pl->side,
                           (const int4 *)Pl->work64, (const int32_t *)Pl->entry_key, (const int32_t *)Pl->entry_src,
                           Pl->key_f64, Pl->nroot, (const float *)Pl->M, (const double *)Pl->Md, Pl->Ld, Pl->partial64,
                           (const int32_t *)Pl->tile_targets);
        HIP_CHECK(hipEventRecord(Pl->ev_join, Pl->side));
    }
    if (Pl->nwork > 0) {
        if (mixed)
            hipLaunchKernelGGL(k_m2l_f16<P>, (int)Pl->nwork, 64 * f16_waves<P>(), 0, s, (const int4 *)Pl->work,
                               (const int32_t *)Pl->entry_key, (const int32_t *)Pl->entry_src,
                               (const uint8_t *)Pl->entry_mask, Pl->key_f16, (const _Float16 *)Pl->Mh,
                               (const _Float16 *)Pl->Ml, (const float *)Pl->Msinv, Pl->L, Pl->partial,
                               (const int32_t *)Pl->tile_targets);
        else if (Pl->key_svd)
            hipLaunchKernelGGL(k_gemm_svd<P>, (int)Pl->nwork, 256, 0, s, (const int4 *)Pl->work,
                               (const int32_t *)Pl->entry_key, (const int32_t *)Pl->entry_src,
                               (const uint8_t *)Pl->entry_mask, Pl->key_svd, (const int32_t *)Pl->key_rank,
                               (const float *)Pl->M, Pl->L, Pl->partial, (const int32_t *)Pl->tile_targets);
        else if (Pl->key_rows)
            hipLaunchKernelGGL((k_gemm<P, false, true, true>), (int)Pl->nwork, 256, 0, s, (const int4 *)Pl->work,
                               (const int32_t *)Pl->entry_key, (const int32_t *)Pl->entry_src,
                               (const uint8_t *)Pl->entry_mask, Pl->key_f32, (const float *)Pl->M, Pl->L, Pl->partial,
                               (const int32_t *)Pl->tile_targets, (const uint32_t *)Pl->key_rows);
        else
            hipLaunchKernelGGL((k_gemm<P, false, true>), (int)Pl->nwork, 256, 0, s, (const int4 *)Pl->work,
                               (const int32_t *)Pl->entry_key, (const int32_t *)Pl->entry_src,
                               (const uint8_t *)Pl->entry_mask, Pl->key_f32, (const float *)Pl->M, Pl->L, Pl->partial,
                               (const int32_t *)Pl->tile_targets);
    }
    // the M2L phase ends after the fixed-order sums of split tiles (and, in mixed precision,
    // after the FP64 root-level M2L on the side stream)
    if (Pl->npartial > 0)
        hipLaunchKernelGGL(k_m2l_reduce, dim3((unsigned)Pl->ntiles, kReduceChunks), 256, 0, s, Pl->ntiles,
                           (const int32_t *)Pl->tile_work,
                           (const int32_t *)Pl->tile_work_idx, (const int4 *)Pl->work, (const float *)Pl->partial,
                           (const int32_t *)Pl->tile_targets, D::KP, Pl->L);
    if (Pl->nruns > 0)
        hipLaunchKernelGGL(k_slot_reduce, (int)std::min<int64_t>(Pl->nruns, 1 << 20), 256, 0, s,
                           Pl->nruns, (const int32_t *)Pl->run_first, (const int32_t *)Pl->run_tgt,
                           (const int64_t *)Pl->slot_pos, (const float *)Pl->partial, D::KP, Pl->L);
    if (root_side) HIP_CHECK(hipStreamWaitEvent(s, Pl->ev_join, 0));
    if (mixed && Pl->partial64)
        hipLaunchKernelGGL(k_m2l64_reduce, dim3((unsigned)Pl->ntiles_root, 16), 256, 0, s, Pl->ntiles_root,
                           (const int32_t *)Pl->tile_work64, (const int32_t *)Pl->tile_work_idx64,
                           (const int4 *)Pl->work64, (const double *)Pl->partial64, (const int32_t *)Pl->tile_targets,
                           D::KP, Pl->Ld);
    ev_rec(Pl, 2 * PH_M2L + 1, s);
    ev_rec(Pl, 2 * PH_L2L, s);
    if (mixed) {
        for (int l = 1; l <= std::min(RL - 1, Pl->max_level); ++l) {
            const int t0 = Pl->l2l.bucket_tile[l * 8], t1 = Pl->l2l.bucket_tile[l * 8 + 8];
            if (t1 > t0)
                hipLaunchKernelGGL((k_gemm64<P, true>), dim3(t1 - t0, kSlabs), 256, 0, s, (const int4 *)Pl->l2l.work + t0,
                                   (const int32_t *)Pl->l2l.entry_key, (const int32_t *)Pl->l2l.entry_src,
                                   T.l2l64_ptrs, Pl->nroot, (const float *)Pl->L, (const double *)Pl->Ld, Pl->Ld,
                                   (double *)nullptr, (const int32_t *)Pl->l2l.tile_targets);
        }
        hipLaunchKernelGGL(k_root_to32, grid1(Pl->nroot * D::KP), 256, 0, s, Pl->nroot, D::KP,
                           (const double *)Pl->Ld, Pl->L);
    }
    for (int l = mixed ? RL : 1; l <= Pl->max_level; ++l) {
        const int t0 = Pl->l2l.bucket_tile[l * 8], t1 = Pl->l2l.bucket_tile[l * 8 + 8];
        if (t1 > t0)
            hipLaunchKernelGGL((k_gemm<P, true, false>), t1 - t0, 256, 0, s, (const int4 *)Pl->l2l.work + t0,
                               (const int32_t *)Pl->l2l.entry_key, (const int32_t *)Pl->l2l.entry_src,
                               (const uint8_t *)nullptr, T.l2l_ptrs, (const float *)Pl->L, Pl->L, (float *)nullptr,
                               (const int32_t *)Pl->l2l.tile_targets);
    }
    ev_rec(Pl, 2 * PH_L2L + 1, s);
    ev_rec(Pl, 2 * PH_L2P, s);
    if (Pl->hess_on)
        hipLaunchKernelGGL(k_l2p_hess<P>, (int)Pl->nleaves, 64, 0, s, (const int32_t *)Pl->leaves, g,
                           (const float4 *)Pl->bodies, (const float *)Pl->L, Pl->far4, Pl->farh);
    else
        hipLaunchKernelGGL(k_l2p<P>, (int)((Pl->n + 255) / 256), 256, 0, s, (const int32_t *)Pl->body_leaf, Pl->n, g,
                           (const float4 *)Pl->bodies, (const float *)Pl->L, Pl->far4);
    ev_rec(Pl, 2 * PH_L2P + 1, s);
}

#define FMM_CASE(PP) case PP: far_field<PP>(Pl, g, s, near); break;

void run_eval(fmm_plan_s *Pl, const float *q, float *phi, float *grad, float *hess, int phases, hipStream_t s,
              const float *dip = nullptr) {
    const int64_t n = Pl->n;
    if (hess && dip) fail(FMM_EINVAL, "internal: a Hessian of dipole sources is not supported");
    Pl->hess_on = hess != nullptr;
    Pl->dip_on = dip != nullptr;
    if (dip && !Pl->dip) {
        hipStream_t keep = Pl->mem.stream;
        Pl->mem.stream = s;
        Pl->dip = Pl->mem.get_n<float4>(n);
        Pl->dipb = Pl->mem.get_n<float4>(n);
        Pl->Mdip = Pl->mem.get_n<float>(3 * Pl->ncells * (int64_t)Pl->KP);
        Pl->mem.stream = keep;
    }
    if (hess && !Pl->farh) {
        hipStream_t keep = Pl->mem.stream;
        Pl->mem.stream = s;
        Pl->farh = Pl->mem.get_n<float>(6 * n);
        Pl->nearh = Pl->mem.get_n<float>(6 * n);
        if (Pl->np2p_part > 0) Pl->p2p_part_h = Pl->mem.get_n<float>(Pl->np2p_part * kP2PThreads * 6);
        Pl->mem.stream = keep;
    }
    Geo g{Pl->c_start, Pl->c_count, Pl->c_level, Pl->c_ix, Pl->c_iy, Pl->c_iz, Pl->c_parent, Pl->c_child0, Pl->c_nchild,
          Pl->x0[0], Pl->x0[1], Pl->x0[2], Pl->k};
    ev_rec(Pl, 2 * PH_TOTAL, s);
    ev_rec(Pl, 2 * PH_PERM, s);
    hipLaunchKernelGGL(k_set_charges, grid1(n), 256, 0, s, q, (const int32_t *)Pl->perm, n, Pl->bodies);
    if (dip) hipLaunchKernelGGL(k_set_dipoles, grid1(n), 256, 0, s, dip, (const int32_t *)Pl->perm, n, Pl->dip);
    ev_rec(Pl, 2 * PH_PERM + 1, s);
    auto near = [&]() { launch_near(Pl, phases, hess != nullptr, s); };
    if ((phases & FMM_FAR) && Pl->nm2l > 0) {
        switch (Pl->p) {
            FMM_CASE(0) FMM_CASE(1) FMM_CASE(2) FMM_CASE(3) FMM_CASE(4) FMM_CASE(5) FMM_CASE(6) FMM_CASE(7)
            FMM_CASE(8) FMM_CASE(9) FMM_CASE(10) FMM_CASE(11) FMM_CASE(12) FMM_CASE(13) FMM_CASE(14)
            FMM_CASE(15) FMM_CASE(16)
            default: fail(FMM_EINVAL, "unsupported order");
        }
    } else {
        near();
        for (int ph = PH_P2M; ph <= PH_L2P; ++ph) { ev_rec(Pl, 2 * ph, s); ev_rec(Pl, 2 * ph + 1, s); }
        fill_f32(reinterpret_cast<float *>(Pl->far4), 0.f, 4 * n, s);
        if (hess) fill_f32(Pl->farh, 0.f, 6 * n, s);
    }
    HIP_CHECK(hipStreamWaitEvent(s, Pl->ev_join, 0));
    ev_rec(Pl, 2 * PH_COMB, s);
    hipLaunchKernelGGL(k_combine, grid1(n), 256, 0, s, (const int32_t *)Pl->iperm, n, (const float4 *)Pl->far4,
                       (const float4 *)Pl->near4, phi, grad);
    if (hess)
        hipLaunchKernelGGL(k_combine_hess, grid1(n), 256, 0, s, (const int32_t *)Pl->iperm, n, (const float *)Pl->farh,
                           (const float *)Pl->nearh, hess);
    ev_rec(Pl, 2 * PH_COMB + 1, s);
    ev_rec(Pl, 2 * PH_TOTAL + 1, s);
    HIP_CHECK(hipGetLastError());
    Pl->ev_valid = Pl->timing;
}

// Adjoint of L(phi, grad phi) with w = dL/dphi and g = dL/d(grad phi) ([n][3]), in two
// evaluations on the frozen plan:
//   dL/dq = Psi,   dL/dx = w E + H g + q grad Psi,
// with E and H the gradient and Hessian of the field of the charges q, and Psi the field of
// the charges w together with dipoles g at the same points.  With K the plan's symmetric
// pair kernel, d(g_i . grad phi_i)/dq_j = g_i . d_1 K(x_i, x_j) = g_i . d_2 K(x_j, x_i): the
// field at x_j of a dipole g_i at x_i (the derivative of its charge's field as x_i moves);
// the same symmetry turns the mixed second derivatives into the gradient of that field.
void run_adjoint_grad(fmm_plan_s *Pl, const float *q, const float *w, const float *g, float *dq, float *dx,
                      hipStream_t s) {
    const int64_t n = Pl->n;
    if (dx && !Pl->tmp_h) {
        hipStream_t keep = Pl->mem.stream;
        Pl->mem.stream = s;
        Pl->tmp_h = Pl->mem.get_n<float>(6 * n);
        Pl->mem.stream = keep;
    }
    if (dx) run_eval(Pl, q, nullptr, Pl->tmp_gfwd, Pl->tmp_h, FMM_ALL, s);
    run_eval(Pl, w, dq ? dq : Pl->tmp_phi, dx ? Pl->tmp_grad : nullptr, nullptr, FMM_ALL, s, g);
    if (dx)
        hipLaunchKernelGGL(k_adjoint_dip_final, grid1(n), 256, 0, s, n, w, (const float *)Pl->tmp_gfwd, q,
                           (const float *)Pl->tmp_grad, (const float *)Pl->tmp_h, g, dx);
    HIP_CHECK(hipGetLastError());
}

void run_adjoint_combine(fmm_plan_s *Pl, const float *w, const float *gphi, const float *q, const float *gpsi, float *dx,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_adjoint_combine, grid1(Pl->n), 256, 0, s, Pl->n, w, gphi, q, gpsi, dx);
    HIP_CHECK(hipGetLastError());
}

}  // namespace fmm
