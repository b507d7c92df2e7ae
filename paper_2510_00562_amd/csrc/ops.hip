// Standalone operators and proximal tools behind geo_apply_op and the
// geo_project_* / geo_prox_l12 entry points. One thread per output element;
// neighbours come through the caches. The solver itself does not use these
// kernels: its fused sweeps (sweep.hip) stage the same stencils in LDS.
#include "solver.hpp"

namespace geo {

namespace {

constexpr int NT = kPointThreads;

struct Cube {
    Dims d;
    __device__ __forceinline__ bool in(int k, int i, int j) const
    {
        return k >= 0 && k < d.n3 && i >= 0 && i < d.n1 && j >= 0 && j < d.n2;
    }
    __device__ __forceinline__ float at(const float *x, int k, int i, int j) const
    {
        return in(k, i, j) ? x[vox(d, k, i, j)] : 0.0f;
    }
};

// ---- differences (Sec. II-A, Neumann boundary) ----
__device__ __forceinline__ float dv(const Cube &c, const float *x, int k, int i, int j)
{
    return i <= c.d.n1 - 2 ? c.at(x, k, i + 1, j) - c.at(x, k, i, j) : 0.0f;
}
__device__ __forceinline__ float dh(const Cube &c, const float *x, int k, int i, int j)
{
    return j <= c.d.n2 - 2 ? c.at(x, k, i, j + 1) - c.at(x, k, i, j) : 0.0f;
}
__device__ __forceinline__ float ds(const Cube &c, const float *x, int k, int i, int j)
{
    return k <= c.d.n3 - 2 ? c.at(x, k + 1, i, j) - c.at(x, k, i, j) : 0.0f;
}
__device__ __forceinline__ float dv_t(const Cube &c, const float *p, int k, int i, int j)
{
    return (i >= 1 ? c.at(p, k, i - 1, j) : 0.0f) - (i <= c.d.n1 - 2 ? c.at(p, k, i, j) : 0.0f);
}
__device__ __forceinline__ float dh_t(const Cube &c, const float *p, int k, int i, int j)
{
    return (j >= 1 ? c.at(p, k, i, j - 1) : 0.0f) - (j <= c.d.n2 - 2 ? c.at(p, k, i, j) : 0.0f);
}
__device__ __forceinline__ float ds_t(const Cube &c, const float *p, int k, int i, int j)
{
    return (k >= 1 ? c.at(p, k - 1, i, j) : 0.0f) - (k <= c.d.n3 - 2 ? c.at(p, k, i, j) : 0.0f);
}
// D D_s (vertical / horizontal) and its adjoint D_s^T D^T
__device__ __forceinline__ float dds_v(const Cube &c, const float *x, int k, int i, int j)
{
    if (k > c.d.n3 - 2 || i > c.d.n1 - 2) return 0.0f;
    return (c.at(x, k + 1, i + 1, j) - c.at(x, k + 1, i, j)) - (c.at(x, k, i + 1, j) - c.at(x, k, i, j));
}
__device__ __forceinline__ float dds_h(const Cube &c, const float *x, int k, int i, int j)
{
    if (k > c.d.n3 - 2 || j > c.d.n2 - 2) return 0.0f;
    return (c.at(x, k + 1, i, j + 1) - c.at(x, k + 1, i, j)) - (c.at(x, k, i, j + 1) - c.at(x, k, i, j));
}
__device__ __forceinline__ float d_t(const Cube &c, const float *pv, const float *ph, int k, int i, int j)
{
    return dv_t(c, pv, k, i, j) + dh_t(c, ph, k, i, j);
}
__device__ __forceinline__ float dds_t(const Cube &c, const float *pv, const float *ph, int k, int i, int j)
{
    float lo = (k >= 1) ? d_t(c, pv, ph, k - 1, i, j) : 0.0f;
    float hi = (k <= c.d.n3 - 2) ? d_t(c, pv, ph, k, i, j) : 0.0f;
    return lo - hi;
}

// ---- Condat's interpolation operators (Sec. II-D) ----
// dual edge fields: vertical on rows 0..N1-2, horizontal on columns 0..N2-2
__device__ __forceinline__ float yvm(const Cube &c, const float *yv, int k, int i, int j)
{
    return (i <= c.d.n1 - 2) ? c.at(yv, k, i, j) : 0.0f;
}
__device__ __forceinline__ float yhm(const Cube &c, const float *yh, int k, int i, int j)
{
    return (j <= c.d.n2 - 2) ? c.at(yh, k, i, j) : 0.0f;
}
// component cmp (0..5 = ud_v, ud_h, lr_v, lr_h, c_v, c_h) of L y
__device__ float l_comp(const Cube &c, const float *yv, const float *yh, int cmp, int k, int i, int j)
{
    const float mv = mask_le(i, c.d.n1), mh = mask_le(j, c.d.n2);
    switch (cmp) {
    case 0: return mv * yvm(c, yv, k, i, j);
    case 1: return mv * 0.25f * (yhm(c, yh, k, i, j) + yhm(c, yh, k, i, j - 1) + yhm(c, yh, k, i + 1, j) + yhm(c, yh, k, i + 1, j - 1));
    case 2: return mh * 0.25f * (yvm(c, yv, k, i, j) + yvm(c, yv, k, i - 1, j) + yvm(c, yv, k, i, j + 1) + yvm(c, yv, k, i - 1, j + 1));
    case 3: return mh * yhm(c, yh, k, i, j);
    case 4: return 0.5f * (yvm(c, yv, k, i, j) + yvm(c, yv, k, i - 1, j));
    default: return 0.5f * (yhm(c, yh, k, i, j) + yhm(c, yh, k, i, j - 1));
    }
}
// w on the ud grid (rows 0..N1-2) and lr grid (cols 0..N2-2)
__device__ __forceinline__ float wud(const Cube &c, const float *w, int k, int i, int j)
{
    return (i <= c.d.n1 - 2) ? c.at(w, k, i, j) : 0.0f;
}
__device__ __forceinline__ float wlr(const Cube &c, const float *w, int k, int i, int j)
{
    return (j <= c.d.n2 - 2) ? c.at(w, k, i, j) : 0.0f;
}
// part (0: vertical, 1: horizontal) of L_g^T w_g for the grids selected by mask
// (bit 0 ud, bit 1 lr, bit 2 c); w points at the 6 planes
__device__ float lt_comp(const Cube &c, const float *w, int64_t N, int gmask, int part, int k, int i, int j)
{
    float acc = 0.0f;
    if (part == 0) {
        if (gmask & 1) acc += wud(c, w + 0 * N, k, i, j);
        if (gmask & 2)
            acc += 0.25f * (wlr(c, w + 2 * N, k, i, j) + wlr(c, w + 2 * N, k, i + 1, j) + wlr(c, w + 2 * N, k, i, j - 1) + wlr(c, w + 2 * N, k, i + 1, j - 1));
        if (gmask & 4) acc += 0.5f * (c.at(w + 4 * N, k, i, j) + c.at(w + 4 * N, k, i + 1, j));
        return mask_le(i, c.d.n1) * acc;
    }
    if (gmask & 2) acc += wlr(c, w + 3 * N, k, i, j);
    if (gmask & 1)
        acc += 0.25f * (wud(c, w + 1 * N, k, i, j) + wud(c, w + 1 * N, k, i, j + 1) + wud(c, w + 1 * N, k, i - 1, j) + wud(c, w + 1 * N, k, i - 1, j + 1));
    if (gmask & 4) acc += 0.5f * (c.at(w + 5 * N, k, i, j) + c.at(w + 5 * N, k, i, j + 1));
    return mask_le(j, c.d.n2) * acc;
}

__global__ __launch_bounds__(NT) void k_apply(int op, int adj, Dims d, const float *in, float *out,
                                              int out_planes)
{
    const Cube c{d};
    const int64_t N = d.plane;
    const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g >= N * out_planes) return;
    const int pl = (int)(g / N);
    const int64_t q = g - (int64_t)pl * N;
    const int j = (int)(q % d.n2);
    const int64_t r = q / d.n2;
    const int i = (int)(r % d.n1), k = (int)(r / d.n1);
    float o = 0.0f;
    if (!adj) {
        switch (op) {
        case GEO_OP_DV: o = dv(c, in, k, i, j); break;
        case GEO_OP_DH: o = dh(c, in, k, i, j); break;
        case GEO_OP_DS: o = ds(c, in, k, i, j); break;
        case GEO_OP_D: o = pl == 0 ? dv(c, in, k, i, j) : dh(c, in, k, i, j); break;
        case GEO_OP_DDS: o = pl == 0 ? dds_v(c, in, k, i, j) : dds_h(c, in, k, i, j); break;
        case GEO_OP_L_UD: o = l_comp(c, in, in + N, 0 + pl, k, i, j); break;
        case GEO_OP_L_LR: o = l_comp(c, in, in + N, 2 + pl, k, i, j); break;
        case GEO_OP_L_C: o = l_comp(c, in, in + N, 4 + pl, k, i, j); break;
        case GEO_OP_L: o = l_comp(c, in, in + N, pl, k, i, j); break;
        case GEO_OP_K: {
            // in: u, s, t, w1 (6), w2 (6); out: y1 (2), y2 (2), y3, y4
            const float *u = in, *s = in + N, *t = in + 2 * N, *w1 = in + 3 * N, *w2 = in + 9 * N;
            if (pl < 2) o = (pl == 0 ? dv(c, u, k, i, j) : dh(c, u, k, i, j)) - lt_comp(c, w1, N, 7, pl, k, i, j);
            else if (pl < 4) o = (pl == 2 ? dds_v(c, u, k, i, j) : dds_h(c, u, k, i, j)) - lt_comp(c, w2, N, 7, pl - 2, k, i, j);
            else if (pl == 4) o = dv(c, t, k, i, j);
            else o = u[q] + s[q] + t[q];
        } break;
        }
    } else {
        switch (op) {
        case GEO_OP_DV: o = dv_t(c, in, k, i, j); break;
        case GEO_OP_DH: o = dh_t(c, in, k, i, j); break;
        case GEO_OP_DS: o = ds_t(c, in, k, i, j); break;
        case GEO_OP_D: o = d_t(c, in, in + N, k, i, j); break;
        case GEO_OP_DDS: o = dds_t(c, in, in + N, k, i, j); break;
        case GEO_OP_L_UD: {
            // in: the 2 planes of the ud grid, placed as planes 0, 1 of a 6-plane view
            o = pl == 0 ? mask_le(i, d.n1) * wud(c, in, k, i, j)
                        : mask_le(j, d.n2) * 0.25f * (wud(c, in + N, k, i, j) + wud(c, in + N, k, i, j + 1) + wud(c, in + N, k, i - 1, j) + wud(c, in + N, k, i - 1, j + 1));
        } break;
        case GEO_OP_L_LR: {
            o = pl == 0 ? mask_le(i, d.n1) * 0.25f * (wlr(c, in, k, i, j) + wlr(c, in, k, i + 1, j) + wlr(c, in, k, i, j - 1) + wlr(c, in, k, i + 1, j - 1))
                        : mask_le(j, d.n2) * wlr(c, in + N, k, i, j);
        } break;
        case GEO_OP_L_C: {
            o = pl == 0 ? mask_le(i, d.n1) * 0.5f * (c.at(in, k, i, j) + c.at(in, k, i + 1, j))
                        : mask_le(j, d.n2) * 0.5f * (c.at(in + N, k, i, j) + c.at(in + N, k, i, j + 1));
        } break;
        case GEO_OP_L: o = lt_comp(c, in, N, 7, pl, k, i, j); break;
        case GEO_OP_K: {
            // in: y1 (2), y2 (2), y3, y4; out: u, s, t, w1 (6), w2 (6)
            const float *y1 = in, *y2 = in + 2 * N, *y3 = in + 4 * N, *y4 = in + 5 * N;
            if (pl == 0) o = d_t(c, y1, y1 + N, k, i, j) + dds_t(c, y2, y2 + N, k, i, j) + y4[q];
            else if (pl == 1) o = y4[q];
            else if (pl == 2) o = dv_t(c, y3, k, i, j) + y4[q];
            else if (pl < 9) o = -l_comp(c, y1, y1 + N, pl - 3, k, i, j);
            else o = -l_comp(c, y2, y2 + N, pl - 9, k, i, j);
        } break;
        }
    }
    out[g] = o;
}

// ---- l2 ball, eq. (23): two-pass FP64 norm, then the scaling ----
__global__ __launch_bounds__(NT) void k_l2_partial(const float *x, const float *cc, int64_t n, double *part)
{
    __shared__ double red[NT / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < n; q += stride) {
        double e = (double)x[q] - (double)cc[q];
        acc += e * e;
    }
    acc = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(NT) void k_l2_final(const double *part, int nb, double *r)
{
    __shared__ double red[NT / 64];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += NT) acc += part[b];
    acc = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) *r = sqrt(acc);
}

__global__ __launch_bounds__(NT) void k_l2_apply(const float *x, const float *cc, int64_t n, double eps,
                                                 const double *r, float *out)
{
    const double rr = *r;
    const bool inside = rr <= eps;
    const double f = inside ? 1.0 : eps / rr;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < n; q += stride)
        out[q] = inside ? x[q] : (float)((double)cc[q] + f * ((double)x[q] - (double)cc[q]));
}

__global__ __launch_bounds__(NT) void k_prox_l12(const float *xa, const float *xb, int64_t n, float g,
                                                 float *oa, float *ob)
{
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < n; q += stride) {
        float a = xa[q], b = xb[q];
        shrink2(a, b, g);
        oa[q] = a;
        ob[q] = b;
    }
}

__global__ __launch_bounds__(NT) void k_box(const float *x, int64_t n, float lo, float hi, float *out)
{
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < n; q += stride) {
        float a = x[q];
        out[q] = a < lo ? lo : (a > hi ? hi : a);
    }
}

int grid_for(int64_t n)
{
    int64_t b = (n + NT - 1) / NT;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

int op_planes(int op, int adj, int *pin, int *pout)
{
    static const int tin[] = {1, 1, 1, 1, 1, 2, 2, 2, 2, 15};
    static const int tout[] = {1, 1, 1, 2, 2, 2, 2, 2, 6, 6};
    if (op < 0 || op > GEO_OP_K) return -1;
    *pin = adj ? tout[op] : tin[op];
    *pout = adj ? tin[op] : tout[op];
    return 0;
}

hipError_t launch_apply_op(int op, int adjoint, const Dims &d, const float *in, float *out, hipStream_t st)
{
    int pin, pout;
    if (op_planes(op, adjoint, &pin, &pout)) return hipErrorInvalidValue;
    const int64_t total = d.plane * pout;
    hipLaunchKernelGGL(k_apply, dim3((unsigned)((total + NT - 1) / NT)), dim3(NT), 0, st, op,
                       adjoint, d, in, out, pout);
    return hipGetLastError();
}

int l2_blocks(int64_t n) { return grid_for(n) > 1024 ? 1024 : grid_for(n); }

hipError_t launch_l2(const float *x, const float *c, int64_t n, double eps, float *out, double *partials,
                     double *r_dev, hipStream_t st)
{
    const int nb = l2_blocks(n);
    hipLaunchKernelGGL(k_l2_partial, dim3(nb), dim3(NT), 0, st, x, c, n, partials);
    hipLaunchKernelGGL(k_l2_final, dim3(1), dim3(NT), 0, st, partials, nb, r_dev);
    hipLaunchKernelGGL(k_l2_apply, dim3(grid_for(n)), dim3(NT), 0, st, x, c, n, eps, r_dev, out);
    return hipGetLastError();
}

hipError_t launch_prox_l12(const float *xa, const float *xb, int64_t n, float gamma, float *oa, float *ob,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_prox_l12, dim3(grid_for(n)), dim3(NT), 0, st, xa, xb, n, gamma, oa, ob);
    return hipGetLastError();
}

hipError_t launch_box(const float *x, int64_t n, float lo, float hi, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_box, dim3(grid_for(n)), dim3(NT), 0, st, x, n, lo, hi, out);
    return hipGetLastError();
}

}  // namespace geo
