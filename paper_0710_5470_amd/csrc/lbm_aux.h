// lbm_aux.h -- initialisation, state exchange and FP64 reductions.
//
// None of these is on the per-step hot path.  Initialisation and state
// exchange always compute in FP64 and round once when storing FP32
// deviations.  Reductions are deterministic: each thread accumulates a fixed
// set of sites in a fixed order, the workgroup combines by a fixed tree, and
// one workgroup sums the per-workgroup partials in index order.
#pragma once

#include "lbm_lattice.h"

namespace lbm {

constexpr int RED_THREADS = 256;

struct Geom {
    int nx, ny, np;    // in-plane x, in-plane y (1 for D2Q9), planes
    long long n;       // sites
    long long stride;  // elements between direction (or component) arrays
};

template <class L> __device__ __forceinline__ void site_coords(const Geom &g, long long s, int &x,
                                                               int &y, int &p)
{
    x = int(s % g.nx);
    long long t = s / g.nx;
    y = int(t % g.ny);
    p = int(t / g.ny);
}

template <class L> __device__ __forceinline__ long long site_index(const Geom &g, int x, int y, int p)
{
    return ((long long)p * g.ny + y) * g.nx + x;
}

// index of r + (sign) e_i
template <class L> __device__ __forceinline__ long long neighbour(const Geom &g, int x, int y, int p,
                                                                  int i, int sign)
{
    int xs = wrap1(x + sign * ox<L>(i), g.nx);
    int ys = L::DIM == 3 ? wrap1(y + sign * oy<L>(i), g.ny) : 0;
    int ps = wrap1(p + sign * op<L>(i), g.np);
    return site_index<L>(g, xs, ys, ps);
}

// f_i(r, 0) = f_i^eq(rho0, rho0 u0) with the stencils applied to rho0; the
// pull layout stores it at r - e_i.
template <class L, int SCHEME, class S>
__global__ void init_kernel(Geom g, Coefs<double> c, const double *__restrict__ rho0,
                            const double *__restrict__ u0, S *__restrict__ dst)
{
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
    double rho = rho0[s];
    double d[3] = {0, 0, 0}, lap = 0;
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        double r = rho0[neighbour<L>(g, x, y, p, i, +1)];
        double cr = coef_grad<L>(c, i) * r;
        d[0] += L::ex[i] * cr;
        d[1] += L::ey[i] * cr;
        d[2] += L::ez[i] * cr;
        lap += coef_lap<L>(c, i) * (r - rho);
    }
    double j[3] = {0, 0, 0};
    if (u0) {
        j[0] = rho * u0[s];
        j[1] = rho * u0[g.stride + s];
        if (L::DIM == 3) j[2] = rho * u0[2 * g.stride + s];
    }
    double feq[L::Q];
    equilibrium<L, SCHEME == SCHEME_EQ>(c, rho - c.shift_sum, j, d, lap, feq);
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        dst[(long long)i * g.stride + neighbour<L>(g, x, y, p, i, -1)] = S(feq[i]);
}

// post-streaming populations f_i(r) = S[i][r - e_i] + s_i, FP64 [q][n]
template <class L, class S>
__global__ void get_state_kernel(Geom g, Coefs<double> c, const S *__restrict__ src,
                                 double *__restrict__ out)
{
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        out[(long long)i * g.stride + s] =
            double(src[(long long)i * g.stride + neighbour<L>(g, x, y, p, i, -1)]) + c.shift[i];
}

template <class L, class S>
__global__ void set_state_kernel(Geom g, Coefs<double> c, const double *__restrict__ in,
                                 S *__restrict__ dst)
{
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        dst[(long long)i * g.stride + neighbour<L>(g, x, y, p, i, -1)] =
            S(in[(long long)i * g.stride + s] - c.shift[i]);
}

// ---- reductions -------------------------------------------------------------

enum RedOp { RED_SUM = 0, RED_MAX = 1, RED_MIN = 2 };

__device__ __forceinline__ double red2(double a, double b, int op)
{
    return op == RED_SUM ? a + b : (op == RED_MAX ? fmax(a, b) : fmin(a, b));
}

// Reduce NV values per thread across the workgroup; thread 0 gets results.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const int (&ops)[NV])
{
    __shared__ double sh[RED_THREADS / 64][NV];
#pragma unroll
    for (int k = 0; k < NV; k++)
        for (int off = 32; off > 0; off >>= 1) v[k] = red2(v[k], __shfl_xor(v[k], off, 64), ops[k]);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) sh[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) {
            double a = sh[0][k];
            for (int w = 1; w < RED_THREADS / 64; w++) a = red2(a, sh[w][k], ops[k]);
            v[k] = a;
        }
    }
}

// Per-direction sums of the stored values: partial[b * Q + i].
template <class L, class S>
__global__ __launch_bounds__(RED_THREADS) void reduce_pops_kernel(Geom g, const S *__restrict__ src,
                                                                  double *__restrict__ partial)
{
    constexpr int Q = L::Q;
    double v[Q];
    int ops[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        v[i] = 0.0;
        ops[i] = RED_SUM;
    }
    long long stride = (long long)gridDim.x * RED_THREADS;
    for (long long s = (long long)blockIdx.x * RED_THREADS + threadIdx.x; s < g.n; s += stride)
#pragma unroll
        for (int i = 0; i < Q; i++) v[i] += double(src[(long long)i * g.stride + s]);
    block_reduce<Q>(v, ops);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < Q; i++) partial[(long long)blockIdx.x * Q + i] = v[i];
}

// Observation fields: [0] max |vel|, [1] max |vel - vel_prev| (0 without a
// previous field), [2] count of bad sites (non-finite, rho <= 0 or
// b rho >= 1), [3] min rho, [4] max rho, [5] sum rho.
constexpr int OBS_NV = 6;

__global__ __launch_bounds__(RED_THREADS) void reduce_obs_kernel(long long n, double b,
                                                                 const double *__restrict__ rho,
                                                                 const double *__restrict__ vel,
                                                                 const double *__restrict__ prev,
                                                                 double *__restrict__ partial)
{
    double v[OBS_NV] = {0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0};
    const int ops[OBS_NV] = {RED_MAX, RED_MAX, RED_SUM, RED_MIN, RED_MAX, RED_SUM};
    long long stride = (long long)gridDim.x * RED_THREADS;
    for (long long s = (long long)blockIdx.x * RED_THREADS + threadIdx.x; s < n; s += stride) {
        double r = rho[s];
        double a = vel ? vel[s] : 0.0, bb = vel ? vel[n + s] : 0.0, cc = vel ? vel[2 * n + s] : 0.0;
        double sp = sqrt(a * a + bb * bb + cc * cc);
        bool bad = !(isfinite(r) && isfinite(sp)) || r <= 0.0 || b * r >= 1.0;
        v[0] = fmax(v[0], sp);
        if (prev) {
            double da = a - prev[s], db = bb - prev[n + s], dc = cc - prev[2 * n + s];
            v[1] = fmax(v[1], sqrt(da * da + db * db + dc * dc));
        }
        v[2] += bad ? 1.0 : 0.0;
        v[3] = fmin(v[3], r);
        v[4] = fmax(v[4], r);
        v[5] += r;
    }
    block_reduce<OBS_NV>(v, ops);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < OBS_NV; k++) partial[(long long)blockIdx.x * OBS_NV + k] = v[k];
}

// One workgroup: combine nblk rows of partials (nv values each, ops per
// column) in row order into out[nv].
// ops: 2 bits per column (RedOp), column k at bits 2k..2k+1.
__global__ __launch_bounds__(RED_THREADS) void finish_kernel(int nblk, int nv,
                                                             unsigned long long ops,
                                                             const double *__restrict__ partial,
                                                             double *__restrict__ out)
{
    // each thread combines a strided subset of rows in increasing order, then
    // the workgroup combines threads in a fixed tree
    for (int k = 0; k < nv; k++) {
        int op = int((ops >> (2 * k)) & 3ull);
        double ident = op == RED_SUM ? 0.0 : (op == RED_MAX ? -INFINITY : INFINITY);
        double a = ident;
        for (int r = threadIdx.x; r < nblk; r += RED_THREADS) a = red2(a, partial[(long long)r * nv + k], op);
        double v1[1] = {a};
        int o1[1] = {op};
        block_reduce<1>(v1, o1);
        if (threadIdx.x == 0) out[k] = v1[0];
        __syncthreads();
    }
}

} // namespace lbm
