// Exact soft-threshold level of the l1-ball projection (constraint sets (16)
// and (17); the paper defers to a fast exact algorithm, any exact projection
// gives the same unique result).
//
// For |z| with FP32 bit patterns P (monotone in the value for non-negative
// floats) the level tau solves f(tau) = radius, f(x) = sum max(|z| - x, 0).
// f is piecewise linear and decreasing, and its value at any bin edge e of a
// histogram over P is exact from suffix counts C and sums S: f(e) = S - e*C.
// A radix search over the 31 pattern bits in three levels (bits 30..20, 19..10,
// 9..0) narrows the bin that holds tau; it stops early when that bin is empty
// (f is linear across it) or holds one value. At the last level every bin is
// one value, so tau = (S_above - radius) / C_above exactly (FP64).
//
// Bin sums are exact: all values of a level-0 bin share one exponent, so their
// sum is an integer sum of 24-bit significands (u64 atomics, order free),
// scaled by a power of two. Histograms are therefore bitwise deterministic.
#include "solver.hpp"

namespace geo {

namespace {

constexpr int kSelThreads = 256;

__device__ __forceinline__ uint32_t abs_bits(float x) { return __float_as_uint(x) & 0x7fffffffu; }

__device__ __forceinline__ uint64_t significand(uint32_t p)
{
    uint32_t e = p >> 23, m = p & 0x7fffffu;
    return e ? (uint64_t)(m | 0x800000u) : (uint64_t)m;
}

// level -> (shift, bins, prefix shift)
__device__ __forceinline__ int lvl_shift(int level) { return level == 0 ? 20 : (level == 1 ? 10 : 0); }
__device__ __forceinline__ int lvl_bins(int level) { return level == 0 ? 2048 : 1024; }

struct ZPtrs {
    const float *z[2];
};

__global__ __launch_bounds__(kSelThreads) void k_select_begin(SelState *sel, int nfields, double r0,
                                                              double r1, Hist *hist,
                                                              const uint32_t *stop)
{
    if (stop && *stop) return;
    const int f = blockIdx.x;
    if (f >= nfields) return;
    for (int b = threadIdx.x; b < kHistBins; b += kSelThreads) {
        hist[f].count[b] = 0u;
        hist[f].msum[b] = 0ull;
    }
    if (threadIdx.x == 0) {
        SelState s;
        s.radius = f == 0 ? r0 : r1;
        s.s_above = 0.0;
        s.c_above = 0ull;
        s.prefix = 0u;
        s.level = 0u;
        s.pad = 0u;
        s.done = s.radius <= 0.0 ? 1u : 0u;
        s.tau = s.radius <= 0.0 ? __longlong_as_double(0x7ff0000000000000ll) : 0.0;
        sel[f] = s;
    }
}

// Histogram of the pattern bits of one radix level, restricted to values
// whose higher bits equal the prefix chosen by the previous levels.
__global__ __launch_bounds__(kSelThreads) void k_hist(ZPtrs zp, int64_t n, const SelState *sel,
                                                      Hist *hist, int level, const uint32_t *stop)
{
    if (stop && *stop) return;
    const int f = blockIdx.y;
    if (sel[f].done || (int)sel[f].level != level) return;
    __shared__ uint32_t cnt[kHistBins];
    __shared__ unsigned long long ms[kHistBins];
    const int bins = lvl_bins(level), shift = lvl_shift(level);
    for (int b = threadIdx.x; b < bins; b += kSelThreads) {
        cnt[b] = 0u;
        ms[b] = 0ull;
    }
    __syncthreads();
    const uint32_t prefix = sel[f].prefix;
    const int pshift = shift + (level == 0 ? 11 : 10);
    const float *z = zp.z[f];
    const int64_t stride = (int64_t)gridDim.x * kSelThreads;
    for (int64_t q = (int64_t)blockIdx.x * kSelThreads + threadIdx.x; q < n; q += stride) {
        uint32_t p = abs_bits(z[q]);
        if (level > 0 && (p >> pshift) != prefix) continue;
        uint32_t b = (p >> shift) & (uint32_t)(bins - 1);
        atomicAdd(&cnt[b], 1u);
        atomicAdd(&ms[b], (unsigned long long)significand(p));
    }
    __syncthreads();
    for (int b = threadIdx.x; b < bins; b += kSelThreads) {
        if (cnt[b]) {
            atomicAdd(&hist[f].count[b], cnt[b]);
            atomicAdd((unsigned long long *)&hist[f].msum[b], ms[b]);
        }
    }
}

// One block per field: pick the bin that holds tau, or finish.
__global__ __launch_bounds__(kSelThreads) void k_select_level(SelState *sel, Hist *hist, int level,
                                                              const uint32_t *stop)
{
    if (stop && *stop) return;
    const int f = blockIdx.x;
    __shared__ SelState s;
    __shared__ double tsum[kSelThreads];
    __shared__ unsigned long long tcnt[kSelThreads];
    __shared__ double sufS[kSelThreads + 1];
    __shared__ unsigned long long sufC[kSelThreads + 1];
    __shared__ int best;
    if (threadIdx.x == 0) {
        s = sel[f];
        best = -1;
    }
    __syncthreads();
    if (s.done || (int)s.level != level) return;
    const int bins = lvl_bins(level), shift = lvl_shift(level);
    const int per = bins / kSelThreads;  // 8 or 4
    const int b0 = threadIdx.x * per;
    // exponent of the values in a bin: level 0 -> from the bin index,
    // deeper levels -> from the prefix
    double bs[8];
    unsigned long long bc[8];
    double ts = 0.0;
    unsigned long long tc = 0ull;
    for (int q = 0; q < per; ++q) {
        int b = b0 + q;
        uint32_t e = level == 0 ? (uint32_t)(b >> 3) : (level == 1 ? (s.prefix >> 3) : (s.prefix >> 13));
        double scale = ldexp(1.0, (int)(e ? e : 1u) - 150);
        bc[q] = hist[f].count[b];
        bs[q] = (double)hist[f].msum[b] * scale;
    }
    // within-thread suffix handled below; thread totals first
    for (int q = 0; q < per; ++q) {
        ts += bs[q];
        tc += bc[q];
    }
    tsum[threadIdx.x] = ts;
    tcnt[threadIdx.x] = tc;
    __syncthreads();
    if (threadIdx.x == 0) {  // fixed-order suffix over threads (deterministic)
        double S = s.s_above;
        unsigned long long C = s.c_above;
        sufS[kSelThreads] = S;
        sufC[kSelThreads] = C;
        for (int t = kSelThreads - 1; t >= 0; --t) {
            S += tsum[t];
            C += tcnt[t];
            sufS[t] = S;
            sufC[t] = C;
        }
    }
    __syncthreads();
    const double radius = s.radius;
    const uint32_t base = level == 0 ? 0u : (s.prefix << (level == 1 ? 20 : 10));
    // walk this thread's bins from the top: S(b), C(b) include bin b
    {
        double S = sufS[threadIdx.x + 1];
        unsigned long long C = sufC[threadIdx.x + 1];
        int mine = -1;
        for (int q = per - 1; q >= 0; --q) {
            int b = b0 + q;
            S += bs[q];
            C += bc[q];
            float eb = __uint_as_float(base | ((uint32_t)b << shift));
            double fb = S - (double)eb * (double)C;
            if (fb >= radius) {
                mine = b;
                break;
            }
        }
        if (mine >= 0) atomicMax(&best, mine);
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    int b = best;
    // Below level 0 the lowest edge of the range has f > radius by
    // construction; FP64 rounding of a differently ordered sum must not turn
    // that into "inside the ball".
    if (b < 0 && level > 0) b = 0;
    // suffix of bins strictly above b
    double Sab = 0.0;
    unsigned long long Cab = 0ull;
    {
        int t = b < 0 ? 0 : b / per;
        Sab = sufS[t + 1];
        Cab = sufC[t + 1];
        for (int bb = t * per + per - 1; bb > b; --bb) {
            uint32_t e = level == 0 ? (uint32_t)(bb >> 3) : (level == 1 ? (s.prefix >> 3) : (s.prefix >> 13));
            Sab += (double)hist[f].msum[bb] * ldexp(1.0, (int)(e ? e : 1u) - 150);
            Cab += hist[f].count[bb];
        }
    }
    SelState o = s;
    if (b < 0) {
        // level 0 only: f(0) = sum |z| < radius: inside the ball
        o.tau = 0.0;
        o.done = 1u;
    } else {
        uint32_t e = level == 0 ? (uint32_t)(b >> 3) : (level == 1 ? (s.prefix >> 3) : (s.prefix >> 13));
        double bsum = (double)hist[f].msum[b] * ldexp(1.0, (int)(e ? e : 1u) - 150);
        unsigned long long bcnt = hist[f].count[b];
        float eb = __uint_as_float(base | ((uint32_t)b << shift));
        double fb = (Sab + bsum) - (double)eb * (double)(Cab + bcnt);
        if (level == 0 && b == 0 && fb <= radius) {
            o.tau = 0.0;  // sum |z| <= radius
            o.done = 1u;
        } else if (fb == radius) {
            o.tau = (double)eb;
            o.done = 1u;
        } else if (bcnt == 0ull || level == 2) {
            // f linear on the bin: every value above tau lies above the bin
            o.tau = (Sab - radius) / (double)Cab;
            o.done = 1u;
        } else if (bcnt == 1ull) {
            // one value a = bsum in the bin
            double a = bsum;
            double t1 = Cab ? (Sab - radius) / (double)Cab : -1.0;
            o.tau = (Cab && t1 >= a) ? t1 : (Sab + a - radius) / (double)(Cab + 1ull);
            o.done = 1u;
        } else {
            o.prefix = (level == 0 ? 0u : (s.prefix << 10)) | (uint32_t)b;
            o.c_above = Cab;
            o.s_above = Sab;
            o.level = (uint32_t)(level + 1);
        }
    }
    sel[f] = o;
}

__global__ __launch_bounds__(kSelThreads) void k_hist_clear(Hist *hist, int nfields,
                                                            const SelState *sel,
                                                            const uint32_t *stop)
{
    if (stop && *stop) return;
    const int f = blockIdx.x;
    if (f >= nfields || sel[f].done) return;
    for (int b = threadIdx.x; b < kHistBins; b += kSelThreads) {
        hist[f].count[b] = 0u;
        hist[f].msum[b] = 0ull;
    }
}

__global__ __launch_bounds__(kSelThreads) void k_soft(const float *x, int64_t n, const SelState *sel,
                                                      float *out)
{
    const double tau = sel->tau;
    const int64_t stride = (int64_t)gridDim.x * kSelThreads;
    for (int64_t q = (int64_t)blockIdx.x * kSelThreads + threadIdx.x; q < n; q += stride) {
        float z = x[q];
        double m = fabs((double)z) - tau;
        out[q] = m > 0.0 ? copysignf((float)m, z) : 0.0f;
    }
}

int hist_blocks(int64_t n)
{
    int b = ceil_div(n, (int64_t)kSelThreads * 16);
    return b < 1 ? 1 : (b > 2048 ? 2048 : b);
}

}  // namespace

// stop may be null (standalone projection)
hipError_t select_begin(SelState *sel, int nfields, double r0, double r1, Hist *hist,
                        const uint32_t *stop, hipStream_t st)
{
    hipLaunchKernelGGL(k_select_begin, dim3(nfields), dim3(kSelThreads), 0, st, sel, nfields, r0,
                       r1, hist, stop);
    return hipGetLastError();
}

hipError_t select_run(const float *z0, const float *z1, int nfields, int64_t n, SelState *sel,
                      Hist *hist, const uint32_t *stop, hipStream_t st)
{
    ZPtrs zp;
    zp.z[0] = z0;
    zp.z[1] = z1;
    const int hb = hist_blocks(n);
    for (int level = 0; level < 3; ++level) {
        hipLaunchKernelGGL(k_hist, dim3(hb, nfields), dim3(kSelThreads), 0, st, zp, n, sel, hist,
                           level, stop);
        hipLaunchKernelGGL(k_select_level, dim3(nfields), dim3(kSelThreads), 0, st, sel, hist,
                           level, stop);
        if (level < 2)
            hipLaunchKernelGGL(k_hist_clear, dim3(nfields), dim3(kSelThreads), 0, st, hist,
                               nfields, sel, stop);
    }
    return hipGetLastError();
}

hipError_t launch_l1_threshold(const float *x, int64_t n, double radius, SelState *sel, Hist *hist,
                               hipStream_t st)
{
    hipError_t e = select_begin(sel, 1, radius, 0.0, hist, nullptr, st);
    if (e != hipSuccess) return e;
    return select_run(x, nullptr, 1, n, sel, hist, nullptr, st);
}

hipError_t launch_soft(const float *x, int64_t n, const SelState *sel, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_soft, dim3(hist_blocks(n)), dim3(kSelThreads), 0, st, x, n, sel, out);
    return hipGetLastError();
}

}  // namespace geo
