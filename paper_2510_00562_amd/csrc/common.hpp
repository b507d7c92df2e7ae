// Device-side helpers shared by the gfx950 kernels of the GeoSSTV solver.
//
// Cube layout is band-sequential: element (i, j, k) of an N1 x N2 x N3 cube at
// (k*N1 + i)*N2 + j, so a wavefront of 64 lanes along j reads 256 contiguous
// bytes of one band row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace geo {

constexpr float kStepU = 1.0f / 13.0f;  // step sizes printed after eq. (24)
constexpr float kStepW = 0.25f;         // w1 and w2
constexpr float kStepT = 1.0f / 3.0f;
constexpr float kStepY = 0.2f;          // y1..y4 (and s has step 1)

// Storage of the dual variables: FP32, or BF16 with FP32 arithmetic.
struct bf16 {
    uint16_t bits;
};

__device__ __forceinline__ float ld(const float *p) { return *p; }
__device__ __forceinline__ float ld(const bf16 *p)
{
    return __uint_as_float(((uint32_t)p->bits) << 16);
}
__device__ __forceinline__ void st(float *p, float x) { *p = x; }
__device__ __forceinline__ void st(bf16 *p, float x)
{
    // round to nearest even; NaN stays NaN
    uint32_t u = __float_as_uint(x);
    uint32_t r = ((u & 0x7fffffffu) > 0x7f800000u) ? (u | 0x00400000u)
                                                   : u + 0x7fffu + ((u >> 16) & 1u);
    bf16 b;
    b.bits = (uint16_t)(r >> 16);
    *p = b;
}

// Pairs stored together: the (vertical, horizontal) components of a dual
// edge field, or the two components of one l_{1,2} group of w.
struct bf16x2 {
    uint32_t bits;  // low half: first component, high half: second
};
template <typename DT> struct PairOf;
template <> struct PairOf<float> { using type = float2; };
template <> struct PairOf<bf16> { using type = bf16x2; };

__device__ __forceinline__ float2 ld2(const float2 *p) { return *p; }
__device__ __forceinline__ float2 ld2(const bf16x2 *p)
{
    const uint32_t b = p->bits;
    return make_float2(__uint_as_float(b << 16), __uint_as_float(b & 0xffff0000u));
}
__device__ __forceinline__ void st2(float2 *p, float2 x) { *p = x; }
__device__ __forceinline__ void st2(bf16x2 *p, float2 x)
{
    bf16 a, b;
    st(&a, x.x);
    st(&b, x.y);
    bf16x2 o;
    o.bits = (uint32_t)a.bits | ((uint32_t)b.bits << 16);
    *p = o;
}

// Stores of results this launch does not read again: with the nontemporal
// hint their lines leave the L2 early and do not push out the halo lines
// that neighbouring tiles still read.
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_nt(float *p, float x)
{
    __builtin_nontemporal_store(x, p);
}
__device__ __forceinline__ void st_nt(float2 *p, float2 x)
{
    f32x2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_nontemporal_store(v, reinterpret_cast<f32x2 *>(p));
}
__device__ __forceinline__ void st_nt(bf16 *p, float x)
{
    bf16 b;
    st(&b, x);
    __builtin_nontemporal_store(b.bits, &p->bits);
}
typedef float f32x4n __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_nt(float4 *p, float4 x)
{
    f32x4n v;
    v.x = x.x;
    v.y = x.y;
    v.z = x.z;
    v.w = x.w;
    __builtin_nontemporal_store(v, reinterpret_cast<f32x4n *>(p));
}
__device__ __forceinline__ void st2_nt(float2 *p, float2 x) { st_nt(p, x); }
__device__ __forceinline__ void st2_nt(bf16x2 *p, float2 x)
{
    bf16 a, b;
    st(&a, x.x);
    st(&b, x.y);
    const uint32_t bits = (uint32_t)a.bits | ((uint32_t)b.bits << 16);
    __builtin_nontemporal_store(bits, &p->bits);
}

// One component (c = 0 first, 1 second) of a stored pair, nontemporal.
__device__ __forceinline__ void st_comp_nt(float2 *p, int c, float x) { st_nt(reinterpret_cast<float *>(p) + c, x); }
__device__ __forceinline__ void st_comp_nt(bf16x2 *p, int c, float x) { st_nt(reinterpret_cast<bf16 *>(p) + c, x); }

// Loads of values no other thread or tile reads (no halo reuse).
__device__ __forceinline__ float ld_nt(const float *p)
{
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ float ld_nt(const bf16 *p)
{
    return __uint_as_float(((uint32_t)__builtin_nontemporal_load(&p->bits)) << 16);
}

struct Dims {
    int n1, n2, n3;
    int64_t plane;  // N = n1*n2*n3 (distance between planes of a field)
};

__device__ __forceinline__ int64_t vox(const Dims &d, int k, int i, int j)
{
    return ((int64_t)k * d.n1 + i) * d.n2 + j;
}

// Masks of the forward differences (Neumann boundary): an edge exists between
// index x and x+1 only for x <= n-2.
__device__ __forceinline__ float mask_le(int x, int n) { return (x >= 0 && x <= n - 2) ? 1.0f : 0.0f; }

// Group shrink of eq. (24) on one pair: scale by max(1 - thr/||(a, b)||, 0),
// with the reciprocal square root instruction (about 1 ulp); a zero pair
// gives rsq = +inf and a zero scale.
__device__ __forceinline__ void shrink2(float &a, float &b, float thr)
{
    const float r = __builtin_amdgcn_rsqf(a * a + b * b);
    const float f = fmaxf(1.0f - thr * r, 0.0f);
    a *= f;
    b *= f;
}

// Wavefront-wide sum of a double (64 lanes).
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Block-wide sum for blocks of up to 1024 threads; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double x, double *lds /* NT/64 */)
{
    x = wave_sum(x);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = x;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += lds[w];
    return s;
}

}  // namespace geo

namespace geo {

// Radix levels of the exact l1-ball threshold search over FP32 bit patterns
// of |z|: level 0 = bits 30..20 (2048 bins), 1 = bits 19..10, 2 = bits 9..0.
__device__ __forceinline__ uint32_t abs_bits(float x) { return __float_as_uint(x) & 0x7fffffffu; }
__device__ __forceinline__ uint64_t significand(uint32_t p)
{
    const uint32_t e = p >> 23, m = p & 0x7fffffu;
    return e ? (uint64_t)(m | 0x800000u) : (uint64_t)m;
}
__device__ __forceinline__ int lvl_shift(int level) { return level == 0 ? 20 : (level == 1 ? 10 : 0); }
__device__ __forceinline__ int lvl_bins(int level) { return level == 0 ? 2048 : 1024; }
// exponent shared by the values of a bin of the given level
__device__ __forceinline__ uint32_t lvl_exponent(int level, uint32_t prefix, int b)
{
    return level == 0 ? (uint32_t)(b >> 3) : (level == 1 ? (prefix >> 3) : (prefix >> 13));
}

// The inputs of the two l1-ball projections (steps 2 and 3 of Alg. 1) and
// y4, written with explicit rounding operations so that every kernel that
// evaluates them (both sweeps and the fallback threshold search) gets
// bit-identical values. y4 is stored as q = 5 y4' - v, the residual of the
// fidelity ball before step 15 rescales it, and read as y4 = a q with a
// device factor a (max(0, 1 - eps/||q||) / 5 after an iteration).
__device__ __forceinline__ float y4_of(float q, float a) { return __fmul_rn(a, q); }
__device__ __forceinline__ float zs_of(float s, float y4) { return __fsub_rn(s, y4); }
// y3m = y3 at (i-1) (0 on the first row), y3c = y3 at i masked by m_v(i),
// step the step size of t (1/3 here; 1/5 for the comparison regularizers)
__device__ __forceinline__ float zt_of(float t, float y3m, float y3c, float y4, float step)
{
    return __fsub_rn(t, __fmul_rn(step, __fadd_rn(__fsub_rn(y3m, y3c), y4)));
}
__device__ __forceinline__ float zt_of(float t, float y3m, float y3c, float y4)
{
    return zt_of(t, y3m, y3c, y4, kStepT);
}

}  // namespace geo
