// The radix levels of the exact l1-ball threshold search, read back from the
// per-level histograms of one field by a single wavefront.
//
// tau solves f(tau) = radius with f(x) = sum max(|z| - x, 0) (the threshold
// of the l1-ball projection of constraint sets (16), (17)). Over the FP32
// bit patterns P of |z| (monotone in the value), three histograms narrow the
// range that holds tau: level 0 bins bits 30..20 (2048 bins), level 1 bits
// 19..10 and level 2 bits 9..0 (1024 bins each) of the values whose higher
// bits equal the bins chosen before. At a bin edge e, f(e) = S(e) - e C(e)
// is exact from the counts and sums of the values at or above e; the level
// picks the highest bin whose lower edge has f >= radius. A level finishes
// the search when that bin is empty or holds one value (f is linear across
// the rest), when its edge gives f = radius exactly, or at level 2, where
// each bin is a single pattern.
//
// Every kernel that needs the outcome (the next level's histogram pass, the
// final pick) evaluates it from the same histograms with the same code: one
// wavefront in a fixed order, independent of the block size, so the FP64
// sums and every decision are bit-identical everywhere.
#pragma once

#include "solver.hpp"

namespace geo {

// Outcome of the radix levels so far for one field.
struct RadixPick {
    double tau;        // final level (done)
    double s_above;    // sum of the values above the current range
    double c_above;    // and their count (exact in FP64)
    double dens;       // values per unit of |z| in the level-0 bin of tau
    uint32_t prefix;   // bits fixed by the levels so far
    int level;         // next level to histogram (3: none)
    int done;
};

__device__ __forceinline__ double bin_scale(uint32_t e) { return ldexp(1.0, (int)(e ? e : 1u) - 150); }

// One level for one field from its histogram staged in LDS (bin sums as
// doubles in bs, counts in bc), by wavefront lanes 0..63 of the caller (every
// lane must call; all lanes return the same result). nb/64 bins per lane,
// lane 0 the top ones.
__device__ __forceinline__ void radix_level_wave(const double *bs, const uint32_t *bc, double radius,
                                                 RadixPick &pk)
{
    const int level = pk.level;
    const int nb = level == 0 ? 2048 : 1024, shift = level == 0 ? 20 : (level == 1 ? 10 : 0);
    const int per = nb / 64;
    const int lane = __lane_id();
    const uint32_t base = level == 0 ? 0u : (pk.prefix << (level == 1 ? 20 : 10));
    const int btop = nb - 1 - per * lane;
    // this lane's bins, top down
    double ls = 0.0, lc = 0.0;
    for (int q = 0; q < per; ++q) {
        ls += bs[btop - q];
        lc += (double)bc[btop - q];
    }
    // inclusive scan over the lanes, lane 0 first
    double xs = ls, xc = lc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double ys = __shfl_up(xs, o, 64), yc = __shfl_up(xc, o, 64);
        if (lane >= o) {
            xs += ys;
            xc += yc;
        }
    }
    // exclusive: the inclusive value of the lane before
    double es = __shfl_up(xs, 1, 64), ec = __shfl_up(xc, 1, 64);
    if (lane == 0) es = ec = 0.0;
    double S = pk.s_above + es, C = pk.c_above + ec;
    const double allS = pk.s_above + __shfl(xs, 63, 64), allC = pk.c_above + __shfl(xc, 63, 64);
    int mine = -1;
    double mS = 0.0, mC = 0.0, mbs = 0.0, mbc = 0.0, mfb = 0.0;
    for (int q = 0; q < per; ++q) {
        const int b = btop - q;
        const double vs = bs[b], vc = (double)bc[b];
        const float eb = __uint_as_float(base | ((uint32_t)b << shift));
        const double fb = (S + vs) - (double)eb * (C + vc);
        if (fb >= radius) {
            mine = b;
            mS = S;  // strictly above bin b
            mC = C;
            mbs = vs;
            mbc = vc;
            mfb = fb;
            break;
        }
        S += vs;
        C += vc;
    }
    // the highest qualifying bin sits in the lowest lane that has one
    const unsigned long long hit = __ballot(mine >= 0);
    int src;
    if (hit) {
        src = __ffsll((long long)hit) - 1;
    } else {
        if (level == 0) {
            // f(0) = sum |z| < radius: inside the ball
            pk.tau = 0.0;
            pk.done = 1;
            pk.level = 3;
            return;
        }
        // FP64 rounding at the lower edge of a deeper range (f there is >=
        // radius by the choice of the range): take bin 0, from the last lane
        src = 63;
        if (lane == 63) {
            mine = 0;
            mbs = bs[0];
            mbc = (double)bc[0];
            mS = allS - mbs;
            mC = allC - mbc;
            mfb = allS - (double)__uint_as_float(base) * allC;
        }
    }
    const int b = __shfl(mine, src, 64);
    mS = __shfl(mS, src, 64);
    mC = __shfl(mC, src, 64);
    mbs = __shfl(mbs, src, 64);
    mbc = __shfl(mbc, src, 64);
    mfb = __shfl(mfb, src, 64);
    const float eb = __uint_as_float(base | ((uint32_t)b << shift));
    if (level == 0) {
        // density of values around tau (sizes the next window); the top bin
        // (patterns of Inf/NaN) never holds tau for finite data
        const double e1 = b + 1 < nb ? (double)__uint_as_float((uint32_t)(b + 1) << shift) : (double)eb;
        pk.dens = e1 > (double)eb ? mbc / (e1 - (double)eb) : 0.0;
    }
    if (mfb == radius) {
        pk.tau = (double)eb;
        pk.done = 1;
    } else if (mbc == 0.0 || level == 2) {
        pk.tau = (mS - radius) / mC;
        pk.done = 1;
    } else if (mbc == 1.0) {
        const double t1 = mC > 0.0 ? (mS - radius) / mC : -1.0;
        pk.tau = (mC > 0.0 && t1 >= mbs) ? t1 : (mS + mbs - radius) / (mC + 1.0);
        pk.done = 1;
    } else {
        pk.prefix = (level == 0 ? 0u : (pk.prefix << 10)) | (uint32_t)b;
        pk.s_above = mS;
        pk.c_above = mC;
    }
    pk.level = pk.done ? 3 : level + 1;
}

// The levels below `upto` (0..3) of field f of a cube, from its histograms
// (hist[level * 2 + f]), by a block of NT threads: every thread stages the
// level's bins into LDS (bs: 2048 doubles, bc: 2048 words), wavefront 0
// decides. Every thread must call; every thread returns the result.
template <int NT>
__device__ RadixPick radix_chain_block(const Hist *hist, int f, double radius, int upto, double *bs,
                                       uint32_t *bc, RadixPick *out)
{
    RadixPick pk = {0.0, 0.0, 0.0, 0.0, 0u, 0, 0};
    while (!pk.done && pk.level < upto) {
        const int level = pk.level, nb = level == 0 ? 2048 : 1024;
        const Hist &h = hist[level * 2 + f];
        for (int b = threadIdx.x; b < nb; b += NT) {
            const uint32_t e = level == 0 ? (uint32_t)(b >> 3) : (level == 1 ? (pk.prefix >> 3) : (pk.prefix >> 13));
            bs[b] = (double)h.msum[b] * bin_scale(e);
            bc[b] = h.count[b];
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            radix_level_wave(bs, bc, radius, pk);
            if (threadIdx.x == 0) *out = pk;
        }
        __syncthreads();
        pk = *out;
        __syncthreads();  // out and the staging are rewritten by the next level
    }
    return pk;
}

// Append val to this block's slice of a field's candidate list. The slot
// comes from an LDS counter (wavefront-aggregated), so sweep A never waits on
// a global atomic; entries past the slice's capacity are counted but
// dropped, which the search detects as an overflow. Every lane of the
// wavefront must call it.
__device__ __forceinline__ void wave_append(bool want, float val, float *slice, uint32_t *lds_count,
                                            int capb)
{
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0u;
    if (lane == leader) base = atomicAdd(lds_count, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    const uint32_t off = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (want && base + off < (uint32_t)capb) slice[base + off] = val;
}

// Candidates a window is widened to when the density of |z| near tau is
// known: the search handles that many in LDS at almost the same cost as a
// few, and a wider window misses less. Once the windows have held for
// kCalmNarrow iterations in a row (tau moves smoothly) the narrower fill
// saves sweep A's appends and the search's bins (256 x 256 x 128: 0.362 ms
// per iteration at 16384 candidates, 0.357 at 8192, 0.3555 at 4096); from
// the start it would miss more.
constexpr double kWindowFill = 16384.0;
constexpr double kWindowFillCalm = 4096.0;
constexpr uint32_t kCalmNarrow = 8;

// Window of |z| that sweep A collects for the next iteration. tau is
// extrapolated from the last levels: quadratically once four are known (the
// levels follow a smooth path after the first iterations, and the quadratic
// error is a fraction of the linear one there), linearly from two or three.
// The half-width is twice the error the same extrapolation made for this
// iteration (plus 5e-5 tau, and never less than the last step plus 2e-4 tau
// when the history is short or the prediction failed). Three times the
// error plus 2e-4 tau held as well in steady state, with windows a third
// wider: the 512 x 512 x 224 search took 89 instead of 51 us. budget > 0
// and the density of |z| near tau known from this iteration: the window is
// widened to hold about `fill` values (the search's cost is flat up to
// there, and a wider window misses less) and narrowed to hold at most about
// `budget` (a window of hundreds of thousands of candidates costs the search
// more than the histogram passes that a miss costs).
__device__ inline void set_window(SelState &o, bool missed, double budget, double fill = kWindowFill)
{
    const double tau = o.tau;
    if (!(tau > 0.0) || !isfinite(tau)) {
        o.win_on = 0u;
        o.tau_prev3 = 0.0;
        o.tau_prev2 = 0.0;
        o.tau_prev = tau;
        return;
    }
    const double t1 = o.tau_prev, t2 = o.tau_prev2, t3 = o.tau_prev3;
    const bool h1 = t1 > 0.0 && isfinite(t1), h2 = h1 && t2 > 0.0 && isfinite(t2);
    const bool h3 = h2 && t3 > 0.0 && isfinite(t3);
    const double step = h1 ? tau - t1 : 0.05 * tau;
    double c = tau + (h1 ? step : 0.0);
    double err = h2 ? fabs(tau - (2.0 * t1 - t2)) : fabs(step);
    if (h3) {
        const double cq = 3.0 * (tau - t1) + t2;
        if (cq > 0.0) {
            c = cq;
            err = fabs(tau - (3.0 * (t1 - t2) + t3));
        }
    }
    double h = 2.0 * err + 5e-5 * tau;
    if (!h2 || missed) h = fmax(h, fabs(step) + 2e-4 * tau);
    if (budget > 0.0 && o.dens > 0.0) {
        // as wide as the search's flat cost allows, narrower than the budget
        h = fmax(h, fill / (2.0 * o.dens));
        h = fmin(h, budget / (2.0 * o.dens));
    }
    double lo = c - h, hi = c + h;
    if (lo < 0.0) lo = 0.0;
    o.win_lo = __double2float_rd(lo);
    o.win_hi = __double2float_ru(hi);
    o.win_on = 1u;
    o.tau_prev3 = h2 ? t2 : 0.0;
    o.tau_prev2 = h1 ? t1 : 0.0;
    o.tau_prev = tau;
}

// Candidate budget of a cube's window: what LDS holds with room for the
// error of the density estimate (20K of the 28K), or for large cubes N/256,
// a streamed search that costs well under the three histogram passes over
// the field that a miss costs.
__host__ __device__ inline double window_budget(int64_t n)
{
    const double b = (double)n / 256.0;
    return b > 20480.0 ? b : 20480.0;
}

}  // namespace geo
