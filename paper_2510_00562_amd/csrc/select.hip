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
#include "radix.hpp"

namespace geo {

namespace {

constexpr int kSelThreads = 256;
constexpr int kHistUnroll = 8;  // values per thread in flight in a histogram pass
// Histogram passes: large blocks, about one per CU and field. Every block
// adds its LDS histogram into the field's global one with atomics, and the
// blocks' atomics on a common bin (values cluster in a few bins) are
// performed one after another: fewer, larger blocks shorten that chain.
constexpr int kHistThreads = 1024;


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
        s.done = s.radius <= 0.0 ? 1u : 0u;
        s.tau = s.radius <= 0.0 ? __longlong_as_double(0x7ff0000000000000ll) : 0.0;
        s.tau_prev = 0.0;
        s.tau_prev2 = 0.0;
        s.tau_prev3 = 0.0;
        s.full = 1u;
        s.win_lo = s.win_hi = 0.f;
        s.win_on = 0u;
        s.cand_count = 0u;
        sel[f] = s;
    }
}

// Values of |z| come either from arrays (standalone projection) or are
// evaluated from the solver state exactly as the sweeps evaluate them.
struct ArraySrc {
    const float *z[2];
    __device__ __forceinline__ void begin() const {}
    __device__ __forceinline__ float get(int f, int64_t q) const { return z[f][q]; }
};

// Histogram of the pattern bits of one radix level, restricted to values
// whose higher bits equal the prefix chosen by the previous levels.
template <typename Src>
__global__ __launch_bounds__(kHistThreads) void k_hist(Src src, int64_t n, const SelState *sel,
                                                      Hist *hist, int level, const uint32_t *stop)
{
    if (stop && *stop) return;
    const int f = blockIdx.y;
    if (sel[f].done || (int)sel[f].level != level) return;
    __shared__ uint32_t cnt[kHistBins];
    __shared__ unsigned long long ms[kHistBins];
    const int bins = lvl_bins(level), shift = lvl_shift(level);
    for (int b = threadIdx.x; b < bins; b += kHistThreads) {
        cnt[b] = 0u;
        ms[b] = 0ull;
    }
    __syncthreads();
    src.begin();
    const uint32_t prefix = sel[f].prefix;
    const int pshift = shift + (level == 0 ? 11 : 10);
    const int64_t stride = (int64_t)gridDim.x * kHistThreads;
    // kHistUnroll loads in flight per thread, then their bins
    for (int64_t q0 = (int64_t)blockIdx.x * kHistThreads + threadIdx.x; q0 < n; q0 += kHistUnroll * stride) {
        uint32_t pv[kHistUnroll];
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) {
            const int64_t q = q0 + u * stride;
            pv[u] = q < n ? abs_bits(src.get(f, q)) : 0u;
        }
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) {
            if (q0 + u * stride >= n) break;
            const uint32_t p = pv[u];
            if (level > 0 && (p >> pshift) != prefix) continue;
            const uint32_t b = (p >> shift) & (uint32_t)(bins - 1);
            atomicAdd(&cnt[b], 1u);
            atomicAdd(&ms[b], (unsigned long long)significand(p));
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < bins; b += kHistThreads) {
        if (cnt[b]) {
            atomicAdd(&hist[f].count[b], cnt[b]);
            atomicAdd((unsigned long long *)&hist[f].msum[b], ms[b]);
        }
    }
}

// One block per field: pick the bin that holds tau, or finish. The block
// stages the level's bins in LDS and one wavefront makes the pick
// (radix_level_wave, the same code as the solver's histogram passes).
__global__ __launch_bounds__(kSelThreads) void k_select_level(SelState *sel, Hist *hist, int level,
                                                              const uint32_t *stop)
{
    if (stop && *stop) return;
    const int f = blockIdx.x;
    __shared__ double bs[kHistBins];
    __shared__ uint32_t bc[kHistBins];
    __shared__ uint32_t fin;
    const SelState s = sel[f];
    if (s.done || (int)s.level != level) return;
    const int nb = lvl_bins(level);
    for (int b = threadIdx.x; b < nb; b += kSelThreads) {
        bs[b] = (double)hist[f].msum[b] * bin_scale(lvl_exponent(level, s.prefix, b));
        bc[b] = hist[f].count[b];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        RadixPick pk = {0.0, s.s_above, (double)s.c_above, 0.0, s.prefix, level, 0};
        radix_level_wave(bs, bc, s.radius, pk);
        if (threadIdx.x == 0) {
            SelState o = s;
            if (pk.done) {
                o.tau = pk.tau;
                o.done = 1u;
                set_window(o, true, 0.0);
            } else {
                o.prefix = pk.prefix;
                o.s_above = pk.s_above;
                o.c_above = (uint64_t)pk.c_above;
                o.level = (uint32_t)(level + 1);
            }
            sel[f] = o;
            fin = o.done;
        }
    }
    __syncthreads();
    // the next level accumulates into a clean histogram
    if (!fin)
        for (int q = threadIdx.x; q < kHistBins; q += kSelThreads) {
            hist[f].count[q] = 0u;
            hist[f].msum[q] = 0ull;
        }
}

// Threshold search over the candidates of the predicted window (one block
// per field). The window holds tau exactly when f(hi) <= radius <= f(lo),
// f(x) = sum max(|z| - x, 0), with f(hi) = S_above - hi C_above and
// f(lo) = f(hi) + sum over candidates of (a - lo) + (hi - lo) C_above.
// Then a radix search over the candidates' bit patterns (levels of at most
// 11 bits aligned to multiples of their width, so no bin straddles an
// exponent and the bin sums stay exact integers) finds tau. Otherwise the
// block prepares the full radix search (level 0) on the whole field.
constexpr int kWinThreads = 1024;
constexpr int kWinBins = 1024;
constexpr int kCandLds = 28672;  // candidates staged in LDS (112 KB); more are streamed
// More candidates than kCandLds are streamed through LDS at every radix
// level, kCandLds at a time. In the pass whose range holds at most kComp of
// them, the ones in range are also compacted into the first kComp entries
// (that pass streams kChunk at a time), and the following levels read only
// those.
constexpr int kChunk = 16384;
constexpr int kComp = kCandLds - kChunk;

// Block-wide exclusive prefix sum (kWinThreads threads, fixed order, so the
// FP64 results are deterministic). wsum: kWinThreads/64 entries of LDS.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T *wsum, T &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    T before = T(0), all = T(0);
    for (int q = 0; q < kWinThreads / 64; ++q) {
        const T v = wsum[q];
        if (q < w) before += v;
        all += v;
    }
    __syncthreads();
    total = all;
    return before + inc - x;
}

// Two block-wide exclusive prefix sums at once (the shuffles of the two
// chains interleave). wsum: 2 * kWinThreads/64 entries of LDS.
// trailing = false leaves out the closing barrier: the caller passes a
// barrier of its own before wsum is written again.
__device__ __forceinline__ void block_exclusive_scan2(double &a, double &b, double *wsum,
                                                      double &ta, double &tb, bool trailing = true)
{
    constexpr int NW = kWinThreads / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double ia = a, ib = b;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double ya = __shfl_up(ia, o, 64), yb = __shfl_up(ib, o, 64);
        if (lane >= o) {
            ia += ya;
            ib += yb;
        }
    }
    if (lane == 63) {
        wsum[w] = ia;
        wsum[NW + w] = ib;
    }
    __syncthreads();
    double ba = 0.0, bb = 0.0, sa = 0.0, sb = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const double va = wsum[q], vb = wsum[NW + q];
        if (q < w) {
            ba += va;
            bb += vb;
        }
        sa += va;
        sb += vb;
    }
    if (trailing) __syncthreads();
    ta = sa;
    tb = sb;
    a = ba + ia - a;
    b = bb + ib - b;
}

// Block-wide sums of three values (fixed order); every thread gets them.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *wsum)
{
    constexpr int NW = kWinThreads / 64;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        wsum[w] = a;
        wsum[NW + w] = b;
        wsum[2 * NW + w] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        a += wsum[q];
        b += wsum[NW + q];
        c += wsum[2 * NW + q];
    }
    __syncthreads();
}

__device__ __forceinline__ double bin_value(unsigned long long msum, uint32_t first_pattern)
{
    const uint32_t e = first_pattern >> 23;
    return (double)msum * ldexp(1.0, (int)(e ? e : 1u) - 150);
}

constexpr double kPrefetchBudgetMB = 96.0;  // of the 256 MB memory-side cache
// Blocks past the search's read sweep B's inputs once, so that sweep B finds
// them in the memory-side cache (the search itself keeps only two CUs per
// cube busy). The values are consumed by an empty asm statement only.
// Every (cube, array) pair is a segment of one flat index space of 16-byte
// words, so a block's loads go out together whatever the number of cubes.
__device__ void prefetch_sweep_b_inputs(const char *table, int stride, int ncubes, int pb, int np)
{
    constexpr int kSeg = kMaxBatch * 5;
    static_assert(kSeg <= kWinThreads, "one segment per thread");
    __shared__ uint32_t seg0[kSeg + 1];  // first flat index of each segment
    __shared__ const uint4 *segp[kSeg];
    __shared__ uint32_t wsu[kWinThreads / 64];
    __shared__ double wsd[3 * (kWinThreads / 64)];
    const int tid = threadIdx.x;
    const uint4 *p = nullptr;
    double bytes = 0.0;
    if (tid < 5 * ncubes) {
        const int c = tid / 5, a = tid % 5;
        const CubeCommon &cc = *reinterpret_cast<const CubeCommon *>(table + (size_t)c * stride);
        const DevScalars *sc = cc.sc;
        if (!idle(sc)) {  // s, t, y3, y4 and the y4 intermediate
            p = reinterpret_cast<const uint4 *>(cc.bin[sc->iter & 1u][a]);
            bytes = (double)cc.bin_bytes[a];
        }
    }
    // at most kPrefetchBudgetMB in all: the leading part of every
    // array, which is what sweep B's first grid-stride rounds read
    double total = bytes, z1 = 0.0, z2 = 0.0;
    block_sum3(total, z1, z2, wsd);
    const double frac = total > 0.0 ? fmin(1.0, kPrefetchBudgetMB * 1048576.0 / total) : 0.0;
    const uint32_t n16 = (uint32_t)(frac * (bytes / 16.0));
    uint32_t all;
    const uint32_t first = block_exclusive_scan<uint32_t>(n16, wsu, all);
    if (tid < kSeg) {
        seg0[tid] = first;
        segp[tid] = p;
    }
    if (tid == 0) seg0[kSeg] = all;
    __syncthreads();
    const int nseg = 5 * ncubes;
    const uint32_t G = (uint32_t)np * kWinThreads;
    for (uint32_t i = (uint32_t)pb * kWinThreads + tid; i < all; i += 4 * G) {
        uint4 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t k = i + u * G;
            x[u] = make_uint4(0u, 0u, 0u, 0u);
            if (k < all) {
                int lo = 0, hi = nseg - 1;  // last segment that starts at or before k
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (seg0[mid] <= k) lo = mid;
                    else hi = mid - 1;
                }
                x[u] = segp[lo][k - seg0[lo]];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) asm volatile("" ::"v"(x[u].x));
    }
}

// One block per (cube, field) of a launch table: block 2c + f; blocks past
// 2 * ncubes prefetch.
__global__ __launch_bounds__(kWinThreads) void k_select_window(const char *table, int stride, int ncubes)
{
    if ((int)blockIdx.x >= 2 * ncubes) {
        prefetch_sweep_b_inputs(table, stride, ncubes, (int)blockIdx.x - 2 * ncubes,
                                (int)gridDim.x - 2 * ncubes);
        return;
    }
    // the launch table through the constant address space (scalar loads)
    const4<CubeCommon> &cc = *(const4<CubeCommon> *)(table + (size_t)(blockIdx.x >> 1) * stride);
    const int f = blockIdx.x & 1;
    DevScalars *sc = cc.sc;
    SelState *sel = sc->sel;
    Hist *hist = cc.hist;
    const double *winpart = cc.winpart;
    const int grid_a = cc.ntiles;  // candidate slices: one per tile
    const float *cand = cc.cand;
    const uint32_t *ccount = cc.ccount;
    const int capb = cc.capt;
    uint32_t *fallback_counter = &sc->fallback;
    __shared__ SelState s;
    __shared__ uint32_t cnt[kWinBins];
    __shared__ unsigned long long ms[kWinBins];
    __shared__ uint32_t pre[kMaxTiles];
    __shared__ float cl[kCandLds + 64];  // staged candidates (+ one wave of slack)
    __shared__ double wsd[3 * (kWinThreads / 64)];
    __shared__ uint32_t wsu[kWinThreads / 64];
    __shared__ double tot[3];
    __shared__ int verdict;  // 0 searching, 1 done, 2 full search needed
    __shared__ int best;
    __shared__ uint32_t ovf, ctot, ncomp, nin;
    __shared__ uint32_t maxown;  // most candidates owned by one thread
    __shared__ uint32_t nbase;
    __shared__ int nshift, nnb;
    __shared__ double nS, nC;
    const int tid = threadIdx.x;
    // Every first read goes out at once: the cube's flags, the field's search
    // state (a word per thread) and sweep A's tile partials and candidate
    // counts (fixed order). A cube that turns out idle has read a few KB for
    // nothing.
    const bool is_idle = idle(sc);
    constexpr int kSelWords = sizeof(SelState) / 4;
    static_assert(sizeof(SelState) % 4 == 0 && kSelWords <= kWinThreads, "search state by words");
    const uint32_t sel_word = tid < kSelWords ? reinterpret_cast<const uint32_t *>(&sel[f])[tid] : 0u;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    uint32_t mine = 0u, cbs[kMaxTiles / kWinThreads];  // this thread's consecutive slices
    bool my_ovf = false;
    const int per = (grid_a + kWinThreads - 1) / kWinThreads;
    for (int b = tid; b < grid_a; b += kWinThreads) {
        const double *w = winpart + ((int64_t)f * grid_a + b) * 3;
        a0 += w[0];
        a1 += w[1];
        a2 += w[2];
    }
#pragma unroll
    for (int q = 0; q < kMaxTiles / kWinThreads; ++q) {
        const int b = per * tid + q;
        uint32_t cb = 0u;
        if (q < per && b < grid_a) {
            cb = ccount[(int64_t)f * grid_a + b];
            if (cb > (uint32_t)capb) {
                my_ovf = true;
                cb = (uint32_t)capb;
            }
        }
        cbs[q] = cb;
        mine += cb;
    }
    if (is_idle) return;
    if (tid < kSelWords) reinterpret_cast<uint32_t *>(&s)[tid] = sel_word;
    if (tid == 0) {
        ovf = 0u;
        maxown = 0u;
        verdict = 0;
    }
    __syncthreads();
    if (my_ovf) atomicOr(&ovf, 1u);  // read after the scans' barriers
    {
        uint32_t mx = mine;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
        if ((tid & 63) == 0) atomicMax(&maxown, mx);  // read after the scans' barriers too
    }
    if (s.radius <= 0.0) {  // zero radius: the ball is {0}
        if (tid == 0) {
            SelState o = s;
            o.tau = __longlong_as_double(0x7ff0000000000000ll);
            o.done = 1u;
            o.full = 0u;
            o.cand_count = 0u;
            o.win_on = 0u;
            sel[f] = o;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < kMaxTiles / kWinThreads; ++q) {
        const int b = per * tid + q;
        if (q < per && b < grid_a) pre[b] = cbs[q];
    }
    uint32_t all_c;
    const uint32_t off = block_exclusive_scan<uint32_t>(mine, wsu, all_c);
    {
        uint32_t acc = off;
        for (int b = per * tid; b < per * tid + per && b < grid_a; ++b) {
            const uint32_t cb = pre[b];
            pre[b] = acc;
            acc += cb;
        }
    }
    block_sum3(a0, a1, a2, wsd);
    const double t0 = a0, t1 = a1, t2 = a2;
    if (tid == 0) {
        ctot = all_c;
        tot[0] = t0;
        tot[1] = t1;
        tot[2] = t2;
        s.cand_count = all_c;
        const double radius = s.radius;
        if (t2 <= radius) {
            verdict = 1;  // inside the ball
            s.tau = 0.0;
        } else if (!s.win_on || ovf || (double)s.win_hi * t0 < t1 - radius) {
            verdict = 2;  // no window, overflow, or tau above the window
        }
    }
    __syncthreads();
    const uint32_t Pa = __float_as_uint(s.win_lo), Pb = __float_as_uint(s.win_hi);
    uint32_t base = 0u;
    int shift = 0, nb = 0;
    double Sab = tot[1], Cab = tot[0];  // count and sum above the current bit range
    if (verdict == 0) {
        const uint32_t span = Pb - Pa;
        const int L = 32 - __clz(span);
        shift = L > 9 ? L - 9 : 0;  // (Pb - base) >> shift < kWinBins
        base = Pa & ~((1u << shift) - 1u);
        nb = (int)((Pb - base) >> shift) + 1;
    }
    int total = (int)ctot;
    // Copy of the candidates at flat positions [c0, c1) (the slices of the
    // tiles one after another, slice b starting at pre[b]) to
    // dst[position - c0]: each thread copies the part of its own slices
    // (those of its `per` consecutive tiles), four loads at a time so that
    // they are in flight together.
    auto copy_own = [&](int c0, int c1, float *dst) {
        for (int b = per * tid; b < per * tid + per && b < grid_a; ++b) {
            const int p0 = (int)pre[b], p1 = b + 1 < grid_a ? (int)pre[b + 1] : total;
            const int lo = p0 > c0 ? p0 : c0, hi = p1 < c1 ? p1 : c1;
            const float *src = cand + ((int64_t)f * grid_a + b) * capb;
            for (int i0 = lo; i0 < hi; i0 += 4) {
                float x[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = i0 + u < hi ? src[i0 + u - p0] : 0.f;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (i0 + u < hi) dst[i0 + u - c0] = x[u];
            }
        }
    };
    // The same copy by wavefronts: wavefront w takes slices w, w + 16, ...;
    // each round of 64 of them reads their bounds with one LDS load per lane
    // and walks them with the bounds read from the lanes (no LDS latency per
    // slice), each lane an asynchronous global-to-LDS load, so that all the
    // loads of the copy are in flight together. Slices outside [c0, c1)
    // cost a few scalar instructions.
    // Which copy: with many small slices (more than 512 tiles, at most 256
    // candidates per thread) the threads' own copies are faster (a stream of
    // 16K candidates from 1792 slices: 8-13 us against 16 us); with large
    // slices they would leave a few threads copying thousands of values one
    // group after another, and the wavefronts copy (the early iterations of
    // 512x512x224, 160K-2.7M candidates: 20% less search time than a walk
    // that read each slice's bounds from LDS).
    auto walk_copy = [&](int c0, int c1, float *dst) {
        const int w = tid >> 6, lane = tid & 63;
        constexpr int NW = kWinThreads / 64;
        for (int b0 = w; b0 < grid_a; b0 += NW * 64) {
            const int bl = b0 + NW * lane;
            const int mp0 = bl < grid_a ? (int)pre[bl] : total;
            const int mp1 = bl + 1 < grid_a ? (int)pre[bl + 1] : total;
            const int nsl = (grid_a - b0 + NW - 1) / NW < 64 ? (grid_a - b0 + NW - 1) / NW : 64;
            for (int l = 0; l < nsl; ++l) {
                const int b = b0 + NW * l;
                const int p0 = __builtin_amdgcn_readlane(mp0, l), p1 = __builtin_amdgcn_readlane(mp1, l);
                const int lo = p0 > c0 ? p0 : c0, hi = p1 < c1 ? p1 : c1;
                const float *src = cand + ((int64_t)f * grid_a + b) * capb + (lo - p0);
                for (int o = 0; o < hi - lo; o += 64)
                    if (o + lane < hi - lo)
                        __builtin_amdgcn_global_load_lds(src + o + lane, dst + (lo - c0) + o, 4, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
    };
    const bool own = grid_a > 512 && maxown <= 256u;
    bool staged = verdict == 0 && total <= kCandLds;
    bool compact = false;  // this level's streaming pass also compacts
    if (staged && own)
        copy_own(0, total, cl);
    else if (staged)
        walk_copy(0, total, cl);
    // bins start empty; each level empties its bins again as it reads them
    for (int b = tid; b < kWinBins; b += kWinThreads) {
        cnt[b] = 0u;
        ms[b] = 0ull;
    }
    if (tid == 0) best = -1;
    __syncthreads();
    // radix levels over the candidates: four barriers each
    for (int level = 0; level < 5 && verdict == 0; ++level) {
        const uint32_t lim = base + ((uint32_t)nb << shift);  // exclusive end of the range
        auto add = [&](uint32_t p) {
            const uint32_t b = (p - base) >> shift;
            atomicAdd(&cnt[b], 1u);
            atomicAdd(&ms[b], (unsigned long long)significand(p));
        };
        if (staged) {
            // four candidates per step, so their LDS reads overlap
            for (int q0 = tid; q0 < total; q0 += 4 * kWinThreads) {
                uint32_t pq[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + u * kWinThreads;
                    pq[u] = q < total ? __float_as_uint(cl[q]) : 0u;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t p = pq[u];
                    if (q0 + u * kWinThreads < total && p >= base && p < lim) add(p);
                }
            }
        } else {
            // stream the candidates through LDS, a chunk at a time in flat
            // order, then every thread bins the chunk
            if (tid == 0) ncomp = 0u;
            // a pass that also compacts keeps the first kComp entries for
            // them; otherwise the chunks take the whole staging area
            float *chunk = compact ? cl + kComp : cl;
            const int csz = compact ? kChunk : kCandLds;
            for (int c0 = 0; c0 < total; c0 += csz) {
                const int c1 = c0 + csz < total ? c0 + csz : total;
                __syncthreads();  // the previous chunk has been binned
                if (own)
                    copy_own(c0, c1, chunk);
                else
                    walk_copy(c0, c1, chunk);
                __syncthreads();
                const int nc = c1 - c0;
                for (int q0 = tid; q0 < nc; q0 += 4 * kWinThreads) {
                    uint32_t pq[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int q = q0 + u * kWinThreads;
                        pq[u] = q < nc ? __float_as_uint(chunk[q]) : 0u;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint32_t p = pq[u];
                        if (q0 + u * kWinThreads < nc && p >= base && p < lim) {
                            add(p);
                            if (compact) {
                                const uint32_t k = atomicAdd(&ncomp, 1u);
                                if (k < (uint32_t)kComp) cl[k] = __uint_as_float(p);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        // one bin per thread: sums strictly above bin b come from a suffix
        // scan (a prefix scan in reversed bin order)
        const int b = kWinBins - 1 - tid;  // reversed
        const bool valid = b < nb;
        const unsigned long long mb = ms[b];
        const uint32_t cb = cnt[b];
        cnt[b] = 0u;  // only this thread reads bin b: empty it for the next level
        ms[b] = 0ull;
        const double bs = valid ? bin_value(mb, base + ((uint32_t)b << shift)) : 0.0;
        const double bc = valid ? (double)cb : 0.0;
        double allS, allC, xS = bs, xC = bc;
        block_exclusive_scan2(xS, xC, wsd, allS, allC, false);
        const double aboveS = Sab + xS;
        const double aboveC = Cab + xC;
        const double radius = s.radius;
        const double S = aboveS + bs, C = aboveC + bc;  // values >= bin b's first edge
        const float eb = valid ? __uint_as_float(base + ((uint32_t)b << shift)) : 0.f;
        const double fb = S - (double)eb * C;
        // highest bin with f(first edge) >= radius: bins run backwards over
        // the lanes, so a wavefront's highest one sits in its lowest lane,
        // and one LDS atomic per wavefront gives the block's (a thousand
        // atomics on one word would queue for microseconds)
        {
            const unsigned long long hit = __ballot(valid && fb >= radius);
            if (hit && (tid & 63) == __ffsll((long long)hit) - 1) atomicMax(&best, b);
        }
        if (level == 0 && tid == 0) {
            // tau below the window: f(lo) < radius (every candidate is >= lo)
            if ((Sab + allS) - (double)s.win_lo * (Cab + allC) < radius) verdict = 2;
        }
        __syncthreads();
        if (verdict == 0) {
            int bb = best;
            if (bb < 0 && level == 0) {
                if (tid == 0) verdict = 2;  // tau below the window
            } else {
                if (bb < 0) bb = 0;  // rounding at the lower edge of a deeper range
                if (b == bb) {
                    const double Sb = aboveS, Cb = aboveC;  // strictly above bin b
                    if (fb == radius) {
                        s.tau = (double)eb;
                        verdict = 1;
                    } else if (bc == 0.0 || shift == 0) {
                        s.tau = (Sb - radius) / Cb;
                        verdict = 1;
                    } else if (bc == 1.0) {
                        const double tl = Cb > 0.0 ? (Sb - radius) / Cb : -1.0;
                        s.tau = (Cb > 0.0 && tl >= bs) ? tl : (Sb + bs - radius) / (Cb + 1.0);
                        verdict = 1;
                    } else {
                        const int ns = shift > 10 ? shift - 10 : 0;
                        nbase = base + ((uint32_t)b << shift);
                        nshift = ns;
                        nnb = 1 << (shift - ns);
                        nS = Sb;
                        nC = Cb;
                        nin = cb;  // candidates in the next level's range
                    }
                }
            }
        }
        __syncthreads();
        if (tid == 0) best = -1;  // every thread has read it
        if (compact) {  // the pass above left the level's range in cl[0, ncomp)
            staged = true;
            compact = false;
            total = (int)ncomp;
        }
        if (verdict == 0) {
            base = nbase;
            shift = nshift;
            nb = nnb;
            Sab = nS;
            Cab = nC;
            compact = !staged && nin <= (uint32_t)kComp;
        }
    }
    if (tid == 0) {
        SelState o = s;
        if (verdict == 1) {
            o.done = 1u;
            o.full = 0u;
            // density of |z| in this iteration's window, for the next one's size
            const double wdt = (double)s.win_hi - (double)s.win_lo;
            o.dens = (s.win_on && wdt > 0.0) ? (double)o.cand_count / wdt : 0.0;
            set_window(o, false, window_budget(cc.d.plane),
                       sc->calm >= kCalmNarrow ? kWindowFillCalm : kWindowFill);
        } else {
            // the radix levels over the whole field, by the histogram passes
            // that follow in this launch slot (fallback.hip)
            o.done = 0u;
            o.full = 1u;
            o.level = 0u;
            o.prefix = 0u;
            o.c_above = 0ull;
            o.s_above = 0.0;
            o.win_on = 0u;
            atomicAdd(fallback_counter, 1u);
            *slot_flags(table, ncubes) = 1u;  // the histogram passes run
        }
        sel[f] = o;
    }
    if (verdict != 1)  // the passes accumulate into clean histograms
        for (int q = tid; q < 3 * kHistBins; q += kWinThreads) {
            Hist &h = hist[(q / kHistBins) * 2 + f];
            h.count[q % kHistBins] = 0u;
            h.msum[q % kHistBins] = 0ull;
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
    // 64 values per thread at most: the block histograms are flushed to
    // global memory with atomics once per block
    int b = ceil_div(n, (int64_t)kHistThreads * 64);
    return b < 1 ? 1 : (b > 256 ? 256 : b);
}

int soft_blocks(int64_t n)
{
    int b = ceil_div(n, (int64_t)kSelThreads * 4);
    return b < 1 ? 1 : (b > 8192 ? 8192 : b);
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
    ArraySrc zp;
    zp.z[0] = z0;
    zp.z[1] = z1;
    const int hb = hist_blocks(n);
    for (int level = 0; level < 3; ++level) {
        hipLaunchKernelGGL(k_hist<ArraySrc>, dim3(hb, nfields), dim3(kHistThreads), 0, st, zp, n,
                           (const SelState *)sel, hist, level, stop);
        hipLaunchKernelGGL(k_select_level, dim3(nfields), dim3(kSelThreads), 0, st, sel, hist,
                           level, stop);
    }
    return hipGetLastError();
}

hipError_t launch_select_window(const void *table, int stride, int ncubes, int prefetch_blocks,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_select_window, dim3(2 * ncubes + prefetch_blocks), dim3(kWinThreads), 0, st,
                       (const char *)table, stride, ncubes);
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
    hipLaunchKernelGGL(k_soft, dim3(soft_blocks(n)), dim3(kSelThreads), 0, st, x, n, sel, out);
    return hipGetLastError();
}

}  // namespace geo
