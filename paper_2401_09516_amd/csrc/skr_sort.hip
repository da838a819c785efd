// Greedy nearest-neighbour sort of the systems (Alg. 1, Sec. 4.1) on gfx950.
//
// 1. Squared distance matrix d2(i, j) = sum_p (P_i[p] - P_j[p])^2 over N x p row-major parameter
//    matrices. Each FP64 difference is rounded as usual, its square is split exactly into two
//    doubles with an FMA, and the squares are accumulated in double-double (error-free sums), then
//    rounded once. The pair is renormalised after every 128-element chunk, which bounds the
//    accumulated error by about p * 128 * 2^-106 relative (~1e-25 at p = 66564), far below half
//    an ulp of the result: the value equals the correctly rounded exact sum except when that sum
//    lies within that distance of a rounding boundary, so the summation order does not matter.
//    One workgroup computes a 16 x 16 tile of pairs over one slice of the parameter index, staging
//    128-element chunks of both row blocks in LDS; only tiles on or above the diagonal are launched.
//    When there are few tiles (few systems, long parameter vectors) the index range is split into
//    slices on their own workgroups; each leaves its renormalised pair, and a second kernel adds
//    the pairs of a tile in slice order with error-free sums (the bound above grows by one 2^-106
//    term per slice) and writes each value to both (i, j) and (j, i).
// 2. One workgroup walks the greedy path: N - 1 steps, each an arg-min over one row of d2 of the
//    unvisited systems, ties to the lowest index, NaN/Inf never preferred (a row with no finite
//    candidate takes the lowest unvisited index).
#include <mutex>

#include "skr_host.hpp"

namespace skr {

constexpr int TS = 16;     // tile side (pairs)
constexpr int PCH = 128;   // parameter chunk staged in LDS

// Slices of the parameter index per tile: enough workgroups to fill the chip, slices of at least
// SLICE_MIN elements.
constexpr long SLICE_MIN = 2048;
constexpr long TARGET_WG = 2048;
long sort_slices(long N, long p) {
    const long nt = (N + TS - 1) / TS;
    const long tiles = nt * (nt + 1) / 2;
    const long by_p = (p + SLICE_MIN - 1) / SLICE_MIN;
    const long by_wg = (TARGET_WG + tiles - 1) / tiles;
    long q = by_p < by_wg ? by_p : by_wg;
    return q < 1 ? 1 : q;
}
// Doubles of slice partials needed for (N, p): zero when one slice per tile suffices.
long sort_part_doubles(long N, long p) {
    const long q = sort_slices(N, p);
    if (q == 1) return 0;
    const long nt = (N + TS - 1) / TS;
    return nt * (nt + 1) / 2 * q * TS * TS * 2;
}

// blockIdx.x = tile, blockIdx.y = slice. part == nullptr: one slice, the value goes to D directly;
// otherwise the renormalised pair (s, lo) goes to part[((tile * nslice + slice) * 256 + thread) * 2].
__global__ __launch_bounds__(TS * TS) void k_sq_dist(const double* __restrict__ P, long N, long p, long slen,
                                                     double* __restrict__ D, double* __restrict__ part) {
#pragma clang fp contract(off)
    // tile index -> (bi, bj) with bi <= bj, row-major over the upper triangle
    const long nt = (N + TS - 1) / TS;
    long tid = blockIdx.x, bi = 0;
    while (tid >= nt - bi) { tid -= nt - bi; ++bi; }
    const long bj = bi + tid;
    __shared__ double Ai[TS * (PCH + 1)];
    __shared__ double Aj[TS * (PCH + 1)];
    const int ti = threadIdx.x / TS, tj = threadIdx.x % TS;
    const long i = bi * TS + ti, j = bj * TS + tj;
    double s = 0.0, lo = 0.0;
    const long p0 = (long)blockIdx.y * slen, p1 = (p0 + slen < p) ? p0 + slen : p;
    for (long e0 = p0; e0 < p1; e0 += PCH) {
        const int len = (int)((p1 - e0) < PCH ? (p1 - e0) : PCH);
        __syncthreads();
        for (int e = threadIdx.x; e < TS * PCH; e += TS * TS) {
            const int r = e / PCH, c = e % PCH;
            const long ri = bi * TS + r, rj = bj * TS + r;
            Ai[r * (PCH + 1) + c] = (ri < N && c < len) ? P[ri * p + e0 + c] : 0.0;
            Aj[r * (PCH + 1) + c] = (rj < N && c < len) ? P[rj * p + e0 + c] : 0.0;
        }
        __syncthreads();
        const double* a = Ai + ti * (PCH + 1);
        const double* b = Aj + tj * (PCH + 1);
        for (int c = 0; c < len; ++c) {
            const double d = a[c] - b[c];
            const double hi = d * d;
            const double he = __builtin_fma(d, d, -hi);   // exact: d*d = hi + he
            // error-free s + hi
            const double t = s + hi;
            const double bb = t - s;
            const double err = (s - (t - bb)) + (hi - bb);
            s = t;
            lo = lo + (err + he);
        }
        // renormalise (s, lo) once per chunk so that |lo| stays below half an ulp of s
        const double t2 = s + lo;
        lo = lo - (t2 - s);
        s = t2;
    }
    if (part) {
        const size_t o = (((size_t)blockIdx.x * gridDim.y + blockIdx.y) * (TS * TS) + threadIdx.x) * 2;
        part[o] = s;
        part[o + 1] = lo;
    } else if (i < N && j < N) {
        const double v = s + lo;
        D[i * N + j] = v;
        D[j * N + i] = v;
    }
}

// One thread per (tile, pair): adds the slices' pairs in slice order, rounds once, writes both halves.
__global__ __launch_bounds__(TS * TS) void k_sq_combine(const double* __restrict__ part, long N, int nslice,
                                                        double* __restrict__ D) {
#pragma clang fp contract(off)
    const long nt = (N + TS - 1) / TS;
    long tid = blockIdx.x, bi = 0;
    while (tid >= nt - bi) { tid -= nt - bi; ++bi; }
    const long bj = bi + tid;
    const int ti = threadIdx.x / TS, tj = threadIdx.x % TS;
    const long i = bi * TS + ti, j = bj * TS + tj;
    double s = 0.0, lo = 0.0;
    for (int q = 0; q < nslice; ++q) {
        const size_t o = (((size_t)blockIdx.x * nslice + q) * (TS * TS) + threadIdx.x) * 2;
        const double hi = part[o], l2 = part[o + 1];
        const double t = s + hi;
        const double bb = t - s;
        const double err = (s - (t - bb)) + (hi - bb);
        s = t;
        lo = lo + (err + l2);
        const double t2 = s + lo;
        lo = lo - (t2 - s);
        s = t2;
    }
    if (i < N && j < N) {
        const double v = s + lo;
        D[i * N + j] = v;
        D[j * N + i] = v;
    }
}

__device__ __forceinline__ bool key_less(double a, long ia, double b, long ib) {
    return a < b || (a == b && ia < ib);
}

constexpr int GW = 256;
constexpr long SORT_NMAX = 262144;   // visited bitmap kept in LDS (32 KB)

__global__ __launch_bounds__(GW) void k_greedy(const double* __restrict__ D, long N, long start,
                                               long long* __restrict__ order, double* __restrict__ dist) {
    __shared__ unsigned visited[SORT_NMAX / 32];
    __shared__ double sk[GW / 64];
    __shared__ long si[GW / 64];
    __shared__ long cur_s;
    const int t = threadIdx.x;
    for (long q = t; q < (N + 31) / 32; q += GW) visited[q] = 0u;
    __syncthreads();
    if (t == 0) {
        visited[start >> 5] |= 1u << (start & 31);
        order[0] = start;
        dist[0] = 0.0;
        cur_s = start;
    }
    __syncthreads();
    for (long step = 1; step < N; ++step) {
        const long cur = cur_s;
        double bk = INFINITY;
        long bi = N;
        for (long jj = t; jj < N; jj += GW) {
            if (visited[jj >> 5] & (1u << (jj & 31))) continue;
            double v = D[cur * N + jj];
            if (!(v < INFINITY)) v = INFINITY;    // NaN and +Inf are never preferred
            if (key_less(v, jj, bk, bi)) { bk = v; bi = jj; }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double ok = __shfl_xor(bk, off, 64);
            const long oi = __shfl_xor(bi, off, 64);
            if (key_less(ok, oi, bk, bi)) { bk = ok; bi = oi; }
        }
        if ((t & 63) == 0) { sk[t >> 6] = bk; si[t >> 6] = bi; }
        __syncthreads();
        if (t == 0) {
            double k0 = sk[0];
            long i0 = si[0];
            for (int q = 1; q < GW / 64; ++q)
                if (key_less(sk[q], si[q], k0, i0)) { k0 = sk[q]; i0 = si[q]; }
            order[step] = i0;
            dist[step] = D[cur * N + i0];
            visited[i0 >> 5] |= 1u << (i0 & 31);
            cur_s = i0;
        }
        __syncthreads();
    }
}

long sort_nmax() { return SORT_NMAX; }

void launch_sort(hipStream_t s, const double* P, long N, long p, long start, double* D, double* part,
                 long long* order, double* dist) {
    const long nt = (N + TS - 1) / TS;
    const long tiles = nt * (nt + 1) / 2;
    const long nslice = sort_slices(N, p);
    const long slen = (p + nslice - 1) / nslice;
    if (tiles > 0 && p > 0) {
        hipLaunchKernelGGL(k_sq_dist, dim3((unsigned)tiles, (unsigned)nslice), dim3(TS * TS), 0, s, P, N, p, slen, D,
                           nslice > 1 ? part : nullptr);
        if (nslice > 1)
            hipLaunchKernelGGL(k_sq_combine, dim3((unsigned)tiles), dim3(TS * TS), 0, s, (const double*)part, N,
                               (int)nslice, D);
    }
    hipLaunchKernelGGL(k_greedy, dim3(1), dim3(GW), 0, s, (const double*)D, N, start, order, dist);
}

// ---------------------------------------------------------------------------------------------
// d2(a, b_c) of a parameter vector against K others for the serving runtime's nearest-chain
// choice, with the same arithmetic as the all-pairs pass: exact squares accumulated in
// double-double, rounded once. Slice q of the index (slen elements) of vector c goes to one
// workgroup: each thread sums a strided subset, the 256 pairs are added in a fixed tree order with
// error-free sums, and the slice's pair is stored; one thread per vector then adds its slices in
// order and writes the rounded value.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void dd_add(double& s, double& lo, double hi, double l2) {
    const double t = s + hi;
    const double bb = t - s;
    const double err = (s - (t - bb)) + (hi - bb);
    s = t;
    lo = lo + (err + l2);
    const double t2 = s + lo;
    lo = lo - (t2 - s);
    s = t2;
}

__device__ __forceinline__ void k_dd_slice_body(const double* __restrict__ a, const double* __restrict__ b, long p,
                                                long slen, double* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double ss[256], sl[256];
    const long p0 = (long)blockIdx.x * slen, p1 = (p0 + slen < p) ? p0 + slen : p;
    double s = 0.0, lo = 0.0;
    int cnt = 0;
    for (long e = p0 + threadIdx.x; e < p1; e += 256) {
        const double d = a[e] - b[e];
        const double hi = d * d;
        const double he = __builtin_fma(d, d, -hi);
        const double t = s + hi;
        const double bb = t - s;
        const double err = (s - (t - bb)) + (hi - bb);
        s = t;
        lo = lo + (err + he);
        if (++cnt == 128) {      // renormalise as the all-pairs pass does per chunk
            const double t2 = s + lo;
            lo = lo - (t2 - s);
            s = t2;
            cnt = 0;
        }
    }
    const double t2 = s + lo;
    lo = lo - (t2 - s);
    s = t2;
    ss[threadIdx.x] = s;
    sl[threadIdx.x] = lo;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double s1 = ss[threadIdx.x], l1 = sl[threadIdx.x];
            dd_add(s1, l1, ss[threadIdx.x + w], sl[threadIdx.x + w]);
            ss[threadIdx.x] = s1;
            sl[threadIdx.x] = l1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss[0];
        part[2 * blockIdx.x + 1] = sl[0];
    }
}

// d2(a, b_c) for K vectors b_c at once: blockIdx.y = c, slice partials at part + 2 * nslice * c.
__global__ __launch_bounds__(256) void k_dd_slice_multi(const double* __restrict__ a, const double* const* bs,
                                                        long p, long slen, double* __restrict__ part) {
    const int c = blockIdx.y;
    k_dd_slice_body(a, bs[c], p, slen, part + 2 * (size_t)gridDim.x * c);
}

// One thread per vector: adds its slices in order and rounds once.
__global__ void k_dd_combine(const double* __restrict__ part, int nslice, int K, double* __restrict__ out) {
#pragma clang fp contract(off)
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= K) return;
    double s = 0.0, lo = 0.0;
    const double* pc = part + 2 * (size_t)nslice * c;
    for (int q = 0; q < nslice; ++q) dd_add(s, lo, pc[2 * q], pc[2 * q + 1]);
    out[c] = s + lo;
}

constexpr long DD_SLICE = 8192;
long dd_slices(long p) { return (p + DD_SLICE - 1) / DD_SLICE; }

// out[c] = d2(a, bs[c]) for c < K (bs: device array of K device pointers); part holds
// 2 * K * dd_slices(p) doubles.
void launch_dd_dist(hipStream_t s, const double* a, const double* const* bs, int K, long p, double* part,
                    double* out) {
    const long ns = dd_slices(p);
    hipLaunchKernelGGL(k_dd_slice_multi, dim3((unsigned)ns, (unsigned)K), dim3(256), 0, s, a, bs, p, DD_SLICE, part);
    hipLaunchKernelGGL(k_dd_combine, dim3((K + 63) / 64), dim3(64), 0, s, (const double*)part, (int)ns, K, out);
}

}  // namespace skr

namespace skr {

// ---------------------------------------------------------------------------------------------
// Allocation-free sort (skr_sort_noalloc): the distance matrix, the slice partials and the order
// and step-distance outputs live in one file-scope device array instead of context buffers. Each
// device holds its own copy; host code reaches it only through the address hipGetSymbolAddress
// returns on that device (the array's name is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------------------------
constexpr long NOALLOC_NMAX = 512;
constexpr size_t NOALLOC_BYTES = (size_t)16 << 20;     // covers every N <= 512 and every p
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAXDEV = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAXDEV] = {};
static int g_scratch_state[NOALLOC_MAXDEV] = {};       // 0 not set up, 1 ready, -1 failed
static hipError_t g_scratch_err[NOALLOC_MAXDEV] = {};

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of scratch a sort of N systems with p parameters uses, and the offsets of its parts.
static size_t noalloc_layout(long N, long p, size_t& off_part, size_t& off_order, size_t& off_dist) {
    off_part = align256((size_t)N * (size_t)N * sizeof(double));
    off_order = off_part + align256((size_t)sort_part_doubles(N, p) * sizeof(double));
    off_dist = off_order + align256((size_t)N * sizeof(long long));
    return off_dist + align256((size_t)N * sizeof(double));
}

// Looks up this device's copy of the scratch array once, with the device current (called by
// skr_ctx_create for the context's device). Returns the runtime's status of the lookup.
hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_state[device] == 0) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void* ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
        g_scratch_err[device] = e;
        if (e == hipSuccess && ptr) {
            g_scratch_ptr[device] = ptr;
            g_scratch_state[device] = 1;
        } else {
            g_scratch_state[device] = -1;
        }
    }
    return g_scratch_err[device];
}

}  // namespace skr

using namespace skr;

extern "C" int skr_sort_noalloc(skr_ctx* ctx, const double* params_dev, int64_t N, int64_t p, int64_t start,
                                int64_t* order_host, double* step_d2_host) {
    if (!ctx) return fail(SKR_EINVAL, "NULL context");
    if (N < 0) return fail(SKR_EINVAL, "N must be >= 0");
    if (N == 0) return SKR_OK;
    if (!order_host) return fail(SKR_EINVAL, "order_host is NULL");
    if (p < 1 || !params_dev) return fail(SKR_EINVAL, "need p >= 1 and params_dev");
    if (start < 0 || start >= N) return fail(SKR_EINVAL, "start %lld out of range", (long long)start);
    if (N > NOALLOC_NMAX)
        return fail(SKR_EINVAL, "skr_sort_noalloc: N = %lld exceeds its limit of %ld systems", (long long)N,
                    NOALLOC_NMAX);
    size_t off_part, off_order, off_dist;
    const size_t need = noalloc_layout((long)N, (long)p, off_part, off_order, off_dist);
    if (need > NOALLOC_BYTES)
        return fail(SKR_EINVAL, "skr_sort_noalloc: N = %lld, p = %lld needs %zu bytes of scratch (limit %zu)",
                    (long long)N, (long long)p, need, NOALLOC_BYTES);
    const int dev = ctx->device;
    if (dev < 0 || dev >= NOALLOC_MAXDEV) return fail(SKR_EINVAL, "device %d out of range", dev);
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (g_scratch_state[dev] == 1) base = g_scratch_ptr[dev];
    }
    if (!base) {
        const hipError_t e = noalloc_setup(dev);
        if (e != hipSuccess) return fail(SKR_EHIP, "scratch lookup on device %d failed: %s", dev, hipGetErrorString(e));
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch_ptr[dev];
    }
    HIPCHK(hipSetDevice(dev));
    unsigned char* b = (unsigned char*)base;
    double* D = (double*)b;
    double* part = (double*)(b + off_part);
    long long* order_d = (long long*)(b + off_order);
    double* dist_d = (double*)(b + off_dist);
    // every entry the kernels read is written earlier in the same call (all N x N distances, the
    // slice partials before they are combined, the whole order), so nothing needs clearing
    launch_sort(ctx->stream, params_dev, (long)N, (long)p, (long)start, D, part, order_d, dist_d);
    HIPLAUNCHCHK();
    HIPCHK(hipMemcpyAsync(order_host, order_d, N * sizeof(long long), hipMemcpyDeviceToHost, ctx->stream));
    if (step_d2_host)
        HIPCHK(hipMemcpyAsync(step_d2_host, dist_d, N * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return SKR_OK;
}

