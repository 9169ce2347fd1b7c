// Device primitives: exclusive scan, LSD radix sort (u64 key, i32 value), fills;
// workspace allocation and error plumbing.
#include "fmm_internal.h"

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

namespace fmm {

[[noreturn]] void fail(fmm_status s, const std::string &msg) { throw Error{s, msg}; }

void check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(FMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Default device memory: a process-wide caching allocator.  Blocks come from
// hipMalloc once and are kept; a block released while work may still be queued is
// reused only by allocations on the same stream (stream order makes that safe);
// blocks released after a synchronisation (plan destroy) serve any stream.
namespace {
struct Block {
    void *p;
    size_t size;
    hipStream_t stream;
    bool any_stream;
    int dev;
};
std::mutex g_cache_mu;
std::multimap<size_t, Block> g_free;                 // size -> free block
std::unordered_map<void *, Block> g_used;            // pointer -> block

size_t round_size(size_t n) {
    if (n <= (1u << 20)) return (n + 511) & ~size_t(511);
    return (n + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
}

void *cache_get(size_t nbytes, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    size_t want = round_size(nbytes);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (auto it = g_free.lower_bound(want); it != g_free.end() && it->first <= want + want / 4; ++it) {
            Block b = it->second;
            if (b.dev != dev || !(b.any_stream || b.stream == s)) continue;
            g_free.erase(it);
            b.stream = s;
            g_used[b.p] = b;
            return b.p;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        // give cached blocks of this device back to the driver and retry once
        (void)hipDeviceSynchronize();
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            for (auto it = g_free.begin(); it != g_free.end();) {
                if (it->second.dev == dev) { (void)hipFree(it->second.p); it = g_free.erase(it); }
                else ++it;
            }
        }
        if (hipMalloc(&p, want) != hipSuccess) return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_used[p] = Block{p, want, s, false, dev};
    return p;
}

void cache_put(void *p, bool synchronized) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_used.find(p);
    if (it == g_used.end()) return;
    Block b = it->second;
    g_used.erase(it);
    b.any_stream = synchronized;
    g_free.emplace(b.size, b);
}
}  // namespace

void *Alloc::get(size_t nbytes) {
    void *p = alloc ? alloc(nbytes, (void *)stream, ctx) : cache_get(nbytes, stream);
    if (!p) fail(FMM_ENOMEM, "device allocation of " + std::to_string(nbytes) + " bytes failed");
    live.push_back(p);
    bytes += (int64_t)nbytes;
    return p;
}

void Alloc::put(void *p) {
    for (size_t i = 0; i < live.size(); ++i)
        if (live[i] == p) {
            if (release) release(p, (void *)stream, ctx);
            else cache_put(p, false);
            live[i] = live.back();
            live.pop_back();
            return;
        }
}

void Alloc::release_all() {
    for (void *p : live) {
        if (release) release(p, (void *)stream, ctx);
        else cache_put(p, true);
    }
    live.clear();
}

// ------------------------------------------------------------------ fills
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f32(float *p, float v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_iota_i32(int32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = (int32_t)i;
}
static int grid_for(int64_t n, int bs = 256) {
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, grid_for(n), 256, 0, s, p, v, n);
}
void fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_f32, grid_for(n), 256, 0, s, p, v, n);
}
void iota_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_iota_i32, grid_for(n), 256, 0, s, p, n);
}

// ------------------------------------------------------------------ scan
// Three-phase exclusive scan: per-block scan (256 threads x 8 items), scan of block
// totals (recursive), add block offsets.
constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_block(const T *in, T *out, T *block_tot, int64_t n) {
    __shared__ T tile[kScanTile];
    __shared__ T part[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
        int64_t g = base + i;
        tile[i] = g < n ? in[g] : T(0);
    }
    __syncthreads();
    T s = 0;
    T loc[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        loc[j] = s;
        s += tile[threadIdx.x * kScanItems + j];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele over the 256 thread totals
    for (int off = 1; off < kScanThreads; off <<= 1) {
        T v = threadIdx.x >= off ? part[threadIdx.x - off] : T(0);
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    T excl = threadIdx.x > 0 ? part[threadIdx.x - 1] : T(0);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) tile[threadIdx.x * kScanItems + j] = loc[j] + excl;
    if (threadIdx.x == kScanThreads - 1 && block_tot) block_tot[blockIdx.x] = part[kScanThreads - 1];
    __syncthreads();
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
        int64_t g = base + i;
        if (g < n) out[g] = tile[i];
    }
}

template <class T>
__global__ void k_scan_add(T *out, const T *block_off, int64_t n) {
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    T add = block_off[blockIdx.x];
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
        int64_t g = base + i;
        if (g < n) out[g] += add;
    }
}

template <class T>
static void scan_rec(const T *in, T *out, int64_t n, Alloc &a, hipStream_t s) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_scan_block<T>, 1, kScanThreads, 0, s, in, out, (T *)nullptr, n);
        return;
    }
    T *tot = a.get_n<T>(nb);
    T *off = a.get_n<T>(nb);
    hipLaunchKernelGGL(k_scan_block<T>, (int)nb, kScanThreads, 0, s, in, out, tot, n);
    scan_rec<T>(tot, off, nb, a, s);
    hipLaunchKernelGGL(k_scan_add<T>, (int)nb, kScanThreads, 0, s, out, (const T *)off, n);
    a.put(tot);
    a.put(off);
}

template <class T>
__global__ void k_total(const T *in, const T *ex, int64_t n, int64_t *tot) {
    *tot = (int64_t)ex[n - 1] + (int64_t)in[n - 1];
}

template <class T>
static int64_t scan_impl(const T *in, T *out, int64_t n, Alloc &a, hipStream_t s) {
    if (n <= 0) return 0;
    scan_rec<T>(in, out, n, a, s);
    int64_t *tot = a.get_n<int64_t>(1);
    hipLaunchKernelGGL(k_total<T>, 1, 1, 0, s, in, (const T *)out, n, tot);
    int64_t r = read_back(tot, s);
    a.put(tot);
    return r;
}

int64_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, Alloc &a, hipStream_t s) {
    return scan_impl<int64_t>(in, out, n, a, s);
}
int64_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, Alloc &a, hipStream_t s) {
    return scan_impl<int32_t>(in, out, n, a, s);
}

// ------------------------------------------------------------------ radix sort
// LSD radix sort, 8-bit digits.  Per pass: (1) per-tile digit histogram, stored
// digit-major so that (2) one exclusive scan gives every (digit, tile) its output
// offset, (3) a stable scatter that ranks equal digits inside a tile with wave
// ballots, keeping the input order among equal digits.
constexpr int kSortThreads = 256, kSortItems = 8, kSortTile = kSortThreads * kSortItems;

__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const uint64_t *keys, int64_t n, int shift, int64_t ntiles,
                                                            int64_t *hist) {
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int i = threadIdx.x; i < kSortTile; i += kSortThreads) {
        int64_t g = base + i;
        if (g < n) atomicAdd(&cnt[(keys[g] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(const uint64_t *kin, const int32_t *vin, uint64_t *kout,
                                                               int32_t *vout, int64_t n, int shift, int64_t ntiles,
                                                               const int64_t *off) {
    __shared__ int64_t base_off[256];
    __shared__ int run[256];
    __shared__ int wcnt[kSortThreads / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    base_off[tid] = off[(int64_t)tid * ntiles + blockIdx.x];
    run[tid] = 0;
    __syncthreads();
    int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        int64_t g = tile0 + (int64_t)r * kSortThreads + tid;
        bool valid = g < n;
        uint64_t key = valid ? kin[g] : 0;
        int32_t val = valid ? vin[g] : 0;
        unsigned d = (unsigned)(key >> shift) & 255u;
        uint64_t mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((d >> b) & 1u);
            mask &= ((d >> b) & 1u) ? bal : ~bal;
        }
        uint64_t lower = mask & ((1ull << lane) - 1ull);
        int rank_in_wave = __popcll(lower);
        if (valid && lower == 0) wcnt[wave][d] = __popcll(mask);   // lowest lane of the digit group
        __syncthreads();
        if (valid) {
            int before = run[d];
            for (int w = 0; w < wave; ++w) before += wcnt[w][d];
            int64_t dst = base_off[d] + before + rank_in_wave;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) add += wcnt[w][tid];
        run[tid] += add;
        __syncthreads();
    }
}

void radix_sort_u64(uint64_t *keys, int32_t *vals, int64_t n, int bits, Alloc &a, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    uint64_t *k2 = a.get_n<uint64_t>(n);
    int32_t *v2 = a.get_n<int32_t>(n);
    int64_t *hist = a.get_n<int64_t>(256 * ntiles);
    int64_t *off = a.get_n<int64_t>(256 * ntiles);
    uint64_t *ki = keys, *ko = k2;
    int32_t *vi = vals, *vo = v2;
    int passes = (bits + 7) / 8;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = 8 * ps;
        hipLaunchKernelGGL(k_sort_hist, (int)ntiles, kSortThreads, 0, s, ki, n, shift, ntiles, hist);
        scan_rec<int64_t>(hist, off, 256 * ntiles, a, s);
        hipLaunchKernelGGL(k_sort_scatter, (int)ntiles, kSortThreads, 0, s, ki, vi, ko, vo, n, shift, ntiles,
                           (const int64_t *)off);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    if (ki != keys) {
        HIP_CHECK(hipMemcpyAsync(keys, ki, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(vals, vi, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    a.put(k2);
    a.put(v2);
    a.put(hist);
    a.put(off);
}

}  // namespace fmm
