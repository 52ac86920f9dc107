// Device-wide primitives for gfx950: integer scans, fills and a stable LSD radix
// sort. All results are deterministic (integer arithmetic, fixed chunking).
#include "common.h"

namespace grass {

namespace {
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;  // 1024

__global__ void k_scan_reduce(const int *__restrict__ in, long long n, int *__restrict__ bsum) {
    __shared__ int red[kScanThreads];
    long long base = (long long)blockIdx.x * kScanTile;
    int s = 0;
    for (int q = 0; q < kScanItems; q++) {
        long long i = base + (long long)q * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kScanThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// exclusive scan of nb block sums by one block of 1024 threads
__global__ void k_scan_bsum(int *__restrict__ bsum, int nb, int *__restrict__ total) {
    __shared__ int sh[1024];
    int t = threadIdx.x;
    int per = (nb + 1023) / 1024;
    int lo = t * per, hi = min(nb, lo + per);
    int s = 0;
    for (int i = lo; i < hi; i++) s += bsum[i];
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int run = sh[t] - s;  // exclusive prefix of this thread's chunk
    for (int i = lo; i < hi; i++) {
        int v = bsum[i];
        bsum[i] = run;
        run += v;
    }
    if (t == 1023 && total) *total = sh[1023];
}

template <bool INCLUSIVE>
__global__ void k_scan_apply(const int *__restrict__ in, int *__restrict__ out, long long n,
                             const int *__restrict__ bsum) {
    __shared__ int sh[kScanThreads];
    long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int q = 0; q < kScanItems; q++) {
        long long i = base + q;
        v[q] = (i < n) ? in[i] : 0;
        s += v[q];
    }
    int t = threadIdx.x;
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int x = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    int run = sh[t] - s + bsum[blockIdx.x];
    for (int q = 0; q < kScanItems; q++) {
        long long i = base + q;
        if (INCLUSIVE) run += v[q];
        if (i < n) out[i] = run;
        if (!INCLUSIVE) run += v[q];
    }
}

template <typename X>
__global__ void k_fill(X *__restrict__ p, long long n, X v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename X>
void fill_impl(X *p, long long n, X v, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill<X>, dim3(blocks), dim3(256), 0, s, p, n, v);
    GR_CHECK_LAUNCH();
}
}  // namespace

void plan_scan(Arena &a, long long n, ScanTmp &t) {
    int nb = div_up(n > 0 ? n : 1, kScanTile);
    t.bsum = a.take<int>(nb + 1);
    t.nblk_cap = nb;
}

static void scan_impl(const int *in, int *out, long long n, int *total, const ScanTmp &t, hipStream_t s,
                      bool inclusive) {
    if (n <= 0) {
        if (total) fill_i32(total, 1, 0, s);
        return;
    }
    int nb = div_up(n, kScanTile);
    require(nb <= t.nblk_cap, GRASS_ERR_OOM, "scan: temp too small");
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, n, t.bsum);
    GR_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(1024), 0, s, t.bsum, nb, total);
    GR_CHECK_LAUNCH();
    if (inclusive)
        hipLaunchKernelGGL(k_scan_apply<true>, dim3(nb), dim3(kScanThreads), 0, s, in, out, n, t.bsum);
    else
        hipLaunchKernelGGL(k_scan_apply<false>, dim3(nb), dim3(kScanThreads), 0, s, in, out, n, t.bsum);
    GR_CHECK_LAUNCH();
}

void scan_excl_i32(const int *in, int *out, long long n, int *total, const ScanTmp &t, hipStream_t s) {
    scan_impl(in, out, n, total, t, s, false);
}
void scan_incl_i32(const int *in, int *out, long long n, const ScanTmp &t, hipStream_t s) {
    scan_impl(in, out, n, nullptr, t, s, true);
}

void fill_i32(int *p, long long n, int v, hipStream_t s) { fill_impl<int>(p, n, v, s); }
void fill_u8(uint8_t *p, long long n, uint8_t v, hipStream_t s) { fill_impl<uint8_t>(p, n, v, s); }
void fill_u32(unsigned *p, long long n, unsigned v, hipStream_t s) { fill_impl<unsigned>(p, n, v, s); }
void fill_f64(double *p, long long n, double v, hipStream_t s) { fill_impl<double>(p, n, v, s); }
void fill_f32(float *p, long long n, float v, hipStream_t s) { fill_impl<float>(p, n, v, s); }

// ------------------------------------------------------------ radix sort
namespace {
constexpr int kSortThreads = 256;  // one item per thread per sub-tile
constexpr int kSortMaxBlocks = 2048;

__global__ void k_radix_hist(const unsigned long long *__restrict__ keys, long long n, int shift, long long chunk,
                             int *__restrict__ hist, int nblk) {
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    long long lo = (long long)blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (long long i = lo + threadIdx.x; i < hi; i += kSortThreads) {
        int d = (int)((keys[i] >> shift) & 255ull);
        atomicAdd(&cnt[d], 1);
    }
    __syncthreads();
    hist[(long long)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void k_radix_scatter(const unsigned long long *__restrict__ kin, const int *__restrict__ vin,
                                unsigned long long *__restrict__ kout, int *__restrict__ vout, long long n,
                                int shift, long long chunk, const int *__restrict__ offs, int nblk) {
    __shared__ int base[256];
    __shared__ int wcnt[4][256];
    __shared__ int wpre[4][256];
    __shared__ int tot[256];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    base[t] = offs[(long long)t * nblk + blockIdx.x];
    long long lo = (long long)blockIdx.x * chunk, hi = min(n, lo + chunk);
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (long long s0 = lo; s0 < hi; s0 += kSortThreads) {
        for (int w = 0; w < 4; w++) wcnt[w][t] = 0;
        __syncthreads();
        long long i = s0 + t;
        bool valid = i < hi;
        unsigned long long key = valid ? kin[i] : 0ull;
        int val = valid ? vin[i] : 0;
        int d = (int)((key >> shift) & 255ull);
        unsigned long long same = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1;
            unsigned long long bb = __ballot(bit);
            same &= bit ? bb : ~bb;
        }
        int rank = __popcll(same & lt);
        if (valid) {
            int leader = 63 - __clzll(same);
            if (lane == leader) wcnt[wave][d] = __popcll(same);
        }
        __syncthreads();
        {
            int run = 0;
            for (int w = 0; w < 4; w++) {
                wpre[w][t] = run;
                run += wcnt[w][t];
            }
            tot[t] = run;
        }
        __syncthreads();
        if (valid) {
            long long pos = (long long)base[d] + wpre[wave][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        base[t] += tot[t];
        __syncthreads();
    }
}

__global__ void k_copy_pairs(const unsigned long long *__restrict__ ks, const int *__restrict__ vs,
                             unsigned long long *__restrict__ kd, int *__restrict__ vd, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}
}  // namespace

void plan_sort(Arena &a, long long n, SortTmp &t) {
    long long cap = n > 0 ? n : 1;
    t.cap = cap;
    t.k2 = a.take<unsigned long long>(cap);
    t.v2 = a.take<int>(cap);
    t.nblk = (int)std::min<long long>(kSortMaxBlocks, std::max<long long>(1, div_up(cap, kSortThreads * 16)));
    t.hist = a.take<int>((size_t)256 * t.nblk);
    plan_scan(a, 256ll * t.nblk, t.scan);
}

void radix_sort_pairs(unsigned long long *keys, int *vals, long long n, int key_bits, const SortTmp &t,
                      hipStream_t s) {
    if (n <= 1) return;
    require(n <= t.cap, GRASS_ERR_OOM, "radix sort: temp too small");
    int nblk = (int)std::min<long long>(t.nblk, div_up(n, kSortThreads));
    long long chunk = ((n + nblk - 1) / nblk + kSortThreads - 1) / kSortThreads * kSortThreads;
    nblk = (int)((n + chunk - 1) / chunk);
    unsigned long long *ka = keys, *kb = t.k2;
    int *va = vals, *vb = t.v2;
    int passes = (key_bits + 7) / 8;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, s, ka, n, shift, chunk, t.hist, nblk);
        GR_CHECK_LAUNCH();
        scan_excl_i32(t.hist, t.hist, 256ll * nblk, nullptr, t.scan, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0, s, ka, va, kb, vb, n, shift, chunk,
                           t.hist, nblk);
        GR_CHECK_LAUNCH();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        int blocks = (int)std::min<long long>(div_up(n, 256), 4096);
        hipLaunchKernelGGL(k_copy_pairs, dim3(blocks), dim3(256), 0, s, ka, va, keys, vals, n);
        GR_CHECK_LAUNCH();
    }
}

}  // namespace grass
