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
    live.emplace_back(p, nbytes);
    bytes += (int64_t)nbytes;
    return p;
}

void Alloc::put(void *p) {
    for (size_t i = 0; i < live.size(); ++i)
        if (live[i].first == p) {
            if (release) release(p, (void *)stream, ctx);
            else cache_put(p, false);
            bytes -= (int64_t)live[i].second;
            live[i] = live.back();
            live.pop_back();
            return;
        }
}

void Alloc::release_all() {
    for (auto &b : live) {
        if (release) release(b.first, (void *)stream, ctx);
        else cache_put(b.first, true);
    }
    live.clear();
    bytes = 0;
}

// ------------------------------------------------------------------ mailbox
namespace {
std::mutex g_mb_mu;
std::vector<Mailbox *> g_mb_free;   // kept for the life of the process
}  // namespace

Mailbox *mailbox_acquire() {
    {
        std::lock_guard<std::mutex> lk(g_mb_mu);
        if (!g_mb_free.empty()) {
            Mailbox *m = g_mb_free.back();
            g_mb_free.pop_back();
            m->upload_used = 0;
            return m;
        }
    }
    void *h = nullptr, *d = nullptr, *f = nullptr, *u = nullptr;
    HIP_CHECK(hipHostMalloc(&h, 64 + Mailbox::kPostBytes,
                            hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable));
    std::memset(h, 0, 64);
    HIP_CHECK(hipHostGetDevicePointer(&d, h, 0));
    HIP_CHECK(hipHostMalloc(&f, Mailbox::kFetchBytes, hipHostMallocPortable));
    HIP_CHECK(hipHostMalloc(&u, Mailbox::kUploadBytes, hipHostMallocPortable));
    Mailbox *m = new Mailbox;
    m->host = static_cast<volatile uint64_t *>(h);
    m->dev = static_cast<uint64_t *>(d);
    m->fetch_host = static_cast<char *>(f);
    m->upload_host = static_cast<char *>(u);
    return m;
}

void mailbox_release(Mailbox *m) {
    if (!m) return;
    std::lock_guard<std::mutex> lk(g_mb_mu);
    g_mb_free.push_back(m);
}

void Mailbox::wait(uint64_t t, hipStream_t s) {
    for (uint64_t it = 1;; ++it) {
        if (__atomic_load_n(&host[0], __ATOMIC_ACQUIRE) == t) return;
        if ((it & 255) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {   // the stream has drained: the ticket must be there
                if (__atomic_load_n(&host[0], __ATOMIC_ACQUIRE) == t) return;
                fail(FMM_EDEVICE, "a device result was not delivered to the host");
            }
            if (e != hipErrorNotReady) check_hip(e, "hipStreamQuery");
        }
    }
}

void Mailbox::upload(void *dst, const void *src, size_t n, hipStream_t s) {
    if (n == 0) return;
    const int64_t off = (upload_used + 255) & ~int64_t(255);
    if (off + (int64_t)n > kUploadBytes) {   // does not fit: a staged copy, completed before returning
        HIP_CHECK(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
        return;
    }
    std::memcpy(upload_host + off, src, n);
    HIP_CHECK(hipMemcpyAsync(dst, upload_host + off, n, hipMemcpyHostToDevice, s));
    upload_used = off + (int64_t)n;
}

const void *Mailbox::fetch(const void *src, size_t n, hipStream_t s) {
    if ((int64_t)n > kFetchBytes) fail(FMM_EUNSUPPORTED, "read-back larger than the mailbox");
    void *dst = fetch_host;
    if (n) HIP_CHECK(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return dst;
}

__global__ void __launch_bounds__(256) k_publish(const uint32_t *src, int64_t words, uint32_t *dst, uint64_t *flag,
                                                 uint64_t ticket) {
    for (int64_t i = threadIdx.x; i < words; i += 256) dst[i] = src[i];
    mailbox_fence();
    __syncthreads();
    if (threadIdx.x == 0) mailbox_post(flag, ticket);
}

void publish(const void *src, int64_t bytes, Mailbox &m, uint64_t ticket, hipStream_t s) {
    if (bytes % 4 != 0 || bytes > Mailbox::kPostBytes) fail(FMM_EINVAL, "publish: bad size");
    hipLaunchKernelGGL(k_publish, 1, 256, 0, s, static_cast<const uint32_t *>(src), bytes / 4,
                       m.data_dev<uint32_t>(), m.flag_dev(), ticket);
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
// Up to kSingleMax values: one workgroup walks the input in tiles of 4096 and carries
// the running total.  Larger inputs: per-block scan (256 threads x 8 items), scan of the
// block totals, add block offsets.  The grand total is written to tot_dst when given,
// followed by a mailbox ticket when flag is given.
constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;
constexpr int kSingleThreads = 1024, kSingleItems = 4, kSingleTile = kSingleThreads * kSingleItems;
constexpr int64_t kSingleMax = 65536;

template <class T>
__global__ void __launch_bounds__(kSingleThreads) k_scan_single(const T *in, T *out, int64_t n, int64_t *tot_dst,
                                                                 uint64_t *flag, uint64_t ticket) {
    __shared__ T wsum[kSingleThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    T carry = 0;
    for (int64_t base = 0; base < n; base += kSingleTile) {
        T v[kSingleItems];
        T sum = 0;
#pragma unroll
        for (int j = 0; j < kSingleItems; ++j) {
            const int64_t g = base + (int64_t)tid * kSingleItems + j;
            v[j] = g < n ? in[g] : T(0);
            sum += v[j];
        }
        T incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const T t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        T wpre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kSingleThreads / 64; ++w) {
            if (w < wave) wpre += wsum[w];
            tot += wsum[w];
        }
        T run = carry + wpre + incl - sum;
#pragma unroll
        for (int j = 0; j < kSingleItems; ++j) {
            const int64_t g = base + (int64_t)tid * kSingleItems + j;
            if (g < n) out[g] = run;
            run += v[j];
        }
        carry += tot;
        __syncthreads();
    }
    if (tid == 0 && tot_dst) {
        *tot_dst = (int64_t)carry;
        if (flag) mailbox_post(flag, ticket);
    }
}

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
__global__ void k_scan_add(T *out, const T *in, const T *block_off, int64_t n, int64_t *tot_dst, uint64_t *flag,
                           uint64_t ticket) {
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    T add = block_off[blockIdx.x];
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
        int64_t g = base + i;
        if (g < n) {
            const T v = out[g] + add;
            out[g] = v;
            if (g == n - 1 && tot_dst) {
                *tot_dst = (int64_t)v + (int64_t)in[g];
                if (flag) mailbox_post(flag, ticket);
            }
        }
    }
}

template <class T>
static void scan_rec(const T *in, T *out, int64_t n, Alloc &a, hipStream_t s, int64_t *tot_dst = nullptr,
                     uint64_t *flag = nullptr, uint64_t ticket = 0) {
    if (n <= kSingleMax) {
        hipLaunchKernelGGL(k_scan_single<T>, 1, kSingleThreads, 0, s, in, out, n, tot_dst, flag, ticket);
        return;
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    T *tot = a.get_n<T>(nb);
    T *off = a.get_n<T>(nb);
    hipLaunchKernelGGL(k_scan_block<T>, (int)nb, kScanThreads, 0, s, in, out, tot, n);
    scan_rec<T>(tot, off, nb, a, s);
    hipLaunchKernelGGL(k_scan_add<T>, (int)nb, kScanThreads, 0, s, out, in, (const T *)off, n, tot_dst, flag, ticket);
    a.put(tot);
    a.put(off);
}

template <class T>
static int64_t scan_impl(const T *in, T *out, int64_t n, Alloc &a, hipStream_t s) {
    if (n <= 0) return 0;
    if (Mailbox *m = a.mb) {
        const uint64_t t = m->next_ticket();
        scan_rec<T>(in, out, n, a, s, m->data_dev<int64_t>(), m->flag_dev(), t);
        m->wait(t, s);
        return m->data_host<int64_t>()[0];
    }
    int64_t *tot = a.get_n<int64_t>(1);
    scan_rec<T>(in, out, n, a, s, tot);
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
void exclusive_scan_i32_to(const int32_t *in, int32_t *out, int64_t n, int64_t *tot_dev, Alloc &a, hipStream_t s) {
    if (n <= 0) {
        fill_i32(reinterpret_cast<int32_t *>(tot_dev), 0, 2, s);
        return;
    }
    scan_rec<int32_t>(in, out, n, a, s, tot_dev);
}
void exclusive_scan_i64_to(const int64_t *in, int64_t *out, int64_t n, int64_t *tot_dev, Alloc &a, hipStream_t s) {
    if (n <= 0) {
        fill_i32(reinterpret_cast<int32_t *>(tot_dev), 0, 2, s);
        return;
    }
    scan_rec<int64_t>(in, out, n, a, s, tot_dev);
}

// ------------------------------------------------------------------ radix sort
// LSD radix sort, 8-bit digits, tiles of 256 x ITEMS keys (ITEMS chosen by the size,
// so that a pass has enough tiles to fill the chip).  Per pass: (1) per-tile digit
// histogram, stored digit-major so that (2) one exclusive scan gives every (digit, tile)
// its output offset, (3) a stable scatter: each wave ranks a contiguous quarter of the
// tile on its own (equal digits in input order, through ballots and per-wave digit
// counters), the quarters are merged by digit in LDS, and the tile is written out (the
// keys, then the values through the same LDS) so that consecutive threads write
// consecutive positions of one digit's run.
constexpr int kSortThreads = 256, kSortWaves = kSortThreads / 64;

template <int kSortItems>
__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const uint64_t *keys, int64_t n, int shift, int64_t ntiles,
                                                            int64_t *hist) {
    constexpr int kSortTile = kSortThreads * kSortItems;
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

template <int kSortItems>
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(const uint64_t *kin, const int32_t *vin, uint64_t *kout,
                                                               int32_t *vout, int64_t n, int shift, int64_t ntiles,
                                                               const int64_t *off) {
    constexpr int kSortTile = kSortThreads * kSortItems;
    // the tile in digit order: keys first, then (reusing the storage) the values, so that
    // the workgroup holds 42 KB of LDS at 4096 keys and three fit on a compute unit
    __shared__ uint64_t sbuf[kSortTile];
    __shared__ uint8_t sdig[kSortTile];   // digit of each position of the ordered tile
    __shared__ int64_t base_off[256];
    __shared__ int wrun[kSortWaves][256];   // per wave: its keys of each digit (then: where they start in the tile)
    __shared__ int wsum[kSortWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    base_off[tid] = off[(int64_t)tid * ntiles + blockIdx.x];
    for (int w = 0; w < kSortWaves; ++w) wrun[w][tid] = 0;
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile, part0 = tile0 + (int64_t)wave * 64 * kSortItems;
    uint64_t key[kSortItems];
    int32_t val[kSortItems];
    int rank[kSortItems];
    int *run = wrun[wave];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t g = part0 + (int64_t)r * 64 + lane;
        const bool valid = g < n;
        key[r] = valid ? kin[g] : 0;
        val[r] = valid ? vin[g] : 0;
        const unsigned d = (unsigned)(key[r] >> shift) & 255u;
        uint64_t mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            mask &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint64_t lower = mask & ((1ull << lane) - 1ull);
        rank[r] = valid ? run[d] + __popcll(lower) : -1;   // rank among this wave's keys of digit d
        // LDS operations of one wave complete in order: every lane has read run[d] above
        // before the lowest lane of the digit group writes it here
        if (valid && lower == 0) run[d] += __popcll(mask);
    }
    __syncthreads();
    // where each wave's keys of each digit start in the digit-sorted tile: digits in
    // order, and inside a digit the waves in order (the input order)
    {
        int c[kSortWaves], v = 0;
        for (int w = 0; w < kSortWaves; ++w) {
            c[w] = wrun[w][tid];
            v += c[w];
        }
        int incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int start = incl - v;
        for (int w = 0; w < wave; ++w) start += wsum[w];
        for (int w = 0; w < kSortWaves; ++w) {
            wrun[w][tid] = start;
            start += c[w];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r)
        if (rank[r] >= 0) {
            rank[r] += run[(unsigned)(key[r] >> shift) & 255u];   // position in the ordered tile
            sbuf[rank[r]] = key[r];
        }
    __syncthreads();
    // wrun[0][d] is now the tile-local start of digit d
    const int cnt = (int)(n - tile0 < kSortTile ? n - tile0 : kSortTile);
    for (int i = tid; i < cnt; i += kSortThreads) {
        const uint64_t k = sbuf[i];
        const unsigned d = (unsigned)(k >> shift) & 255u;
        sdig[i] = (uint8_t)d;
        kout[base_off[d] + (i - wrun[0][d])] = k;
    }
    __syncthreads();
    int32_t *sv = reinterpret_cast<int32_t *>(sbuf);
#pragma unroll
    for (int r = 0; r < kSortItems; ++r)
        if (rank[r] >= 0) sv[rank[r]] = val[r];
    __syncthreads();
    for (int i = tid; i < cnt; i += kSortThreads) {
        const unsigned d = sdig[i];
        vout[base_off[d] + (i - wrun[0][d])] = sv[i];
    }
}

template <int kSortItems>
static void radix_passes(uint64_t *&ki, int32_t *&vi, uint64_t *&ko, int32_t *&vo, int64_t n, int passes, Alloc &a,
                         hipStream_t s) {
    constexpr int kSortTile = kSortThreads * kSortItems;
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    int64_t *hist = a.get_n<int64_t>(256 * ntiles);
    int64_t *off = a.get_n<int64_t>(256 * ntiles);
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 8 * ps;
        hipLaunchKernelGGL(k_sort_hist<kSortItems>, (int)ntiles, kSortThreads, 0, s, ki, n, shift, ntiles, hist);
        scan_rec<int64_t>(hist, off, 256 * ntiles, a, s);
        hipLaunchKernelGGL(k_sort_scatter<kSortItems>, (int)ntiles, kSortThreads, 0, s, ki, vi, ko, vo, n, shift,
                           ntiles, (const int64_t *)off);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    a.put(hist);
    a.put(off);
}

void radix_sort_u64(uint64_t *&keys, int32_t *&vals, int64_t n, int bits, Alloc &a, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    uint64_t *k2 = a.get_n<uint64_t>(n);
    int32_t *v2 = a.get_n<int32_t>(n);
    uint64_t *ki = keys, *ko = k2;
    int32_t *vi = vals, *vo = v2;
    const int passes = (bits + 7) / 8;
    // tiles of 4096 keys from 2^23 keys on, 2048 from 2^22, else 1024: at least ~2048 tiles
    // per pass where the size allows, and long per-digit runs in the scatter
    if (n >= (int64_t(1) << 23)) radix_passes<16>(ki, vi, ko, vo, n, passes, a, s);
    else if (n >= (int64_t(1) << 22)) radix_passes<8>(ki, vi, ko, vo, n, passes, a, s);
    else radix_passes<4>(ki, vi, ko, vo, n, passes, a, s);
    if (ki != keys) {   // odd number of passes: the result is in the second pair
        a.put(keys);
        a.put(vals);
        keys = ki;
        vals = vi;
    } else {
        a.put(k2);
        a.put(v2);
    }
}

}  // namespace fmm
