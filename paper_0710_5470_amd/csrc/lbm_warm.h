// lbm_warm.h -- device side of the warm start's data preparation: network
// input features and the projection of a network prediction onto a valid
// initial field (square symmetry, the cold start's mass, zero momentum).
#pragma once

#include <hip/hip_runtime.h>

namespace lbmwarm {

constexpr int WARM_THREADS = 1024;
constexpr int FEAT_C = 16;  // padded input channels

// Features of problem k at site s: channels 0..4 are per-problem constants
// (host-normalised), channel 5 the normalised initial density, the rest 0.
__global__ void warm_features_kernel(int nprob, int side, const double *__restrict__ consts,
                                     const double *__restrict__ rho0, double rho_mean, double rho_scale,
                                     float *__restrict__ x)
{
    const long long n = (long long)side * side;
    const long long total = n * nprob;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const long long k = q / n;
        float v[FEAT_C];
#pragma unroll
        for (int c = 0; c < FEAT_C; c++) v[c] = 0.0f;
#pragma unroll
        for (int c = 0; c < 5; c++) v[c] = float(consts[k * 5 + c]);
        v[5] = float((rho0[q] - rho_mean) / rho_scale);
        float4 *o = reinterpret_cast<float4 *>(x + q * FEAT_C);
#pragma unroll
        for (int c = 0; c < FEAT_C / 4; c++) o[c] = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
    }
}

// Training target of problem k at site s: channel 0 = (rho - rho0) / s_rho,
// channels 1, 2 = (u_x, u_y) / s_u (vel is [3][ntot]), the rest 0.
__global__ void warm_targets_kernel(long long ntot, const double *__restrict__ rho,
                                    const double *__restrict__ rho0, const double *__restrict__ vel,
                                    double s_rho, double s_u, float *__restrict__ y)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < ntot;
         q += (long long)gridDim.x * blockDim.x) {
        float v[FEAT_C];
#pragma unroll
        for (int c = 0; c < FEAT_C; c++) v[c] = 0.0f;
        v[0] = float((rho[q] - rho0[q]) / s_rho);
        v[1] = float(vel[q] / s_u);
        v[2] = float(vel[ntot + q] / s_u);
        float4 *o = reinterpret_cast<float4 *>(y + q * FEAT_C);
#pragma unroll
        for (int c = 0; c < FEAT_C / 4; c++) o[c] = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
    }
}

// Fixed-order block sum of NV doubles (deterministic for a fixed blockDim).
template <int NV> __device__ void block_sum(double (&v)[NV])
{
    __shared__ double part[NV][WARM_THREADS / 64];
#pragma unroll
    for (int i = 0; i < NV; i++) {
        double a = v[i];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        v[i] = a;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; i++) part[i][wv] = v[i];
    }
    __syncthreads();
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; i++) {
        double a = 0.0;
        for (int w = 0; w < nw; w++) a += part[i][w];
        v[i] = a;
    }
    __syncthreads();  // part is reused by the next call
}

// One workgroup per problem (a side x side D2Q9 lattice, drop centred on the
// node (side/2, side/2)).  pred: [nprob][side][side][cpad] network output,
// channel 0 = (rho - rho0) / s_rho, channels 1, 2 = u / s_u.
//   1. decode and, if sym, average over the eight symmetries g of the square
//      about the centre: rho(p) = mean_g rho(g p), u(p) = mean_g M_g^T u(g p)
//      (M_g the matrix of g), so the field has the drop's own symmetry;
//   2. add the uniform density that restores the cold start's mass, clamp
//      to [rho_lo, rho_hi];
//   3. subtract the mass-weighted mean velocity (zero momentum).
// A problem with any non-finite prediction gets rho0 and u = 0.
__global__ __launch_bounds__(WARM_THREADS) void warm_project_kernel(
    int side, int cpad, const float *__restrict__ pred, const double *__restrict__ rho0, double s_rho,
    double s_u, int with_u, int sym, double rho_lo, double rho_hi, double *__restrict__ rho_out,
    double *__restrict__ u_out, long long ntot)
{
    const int k = blockIdx.x;
    const int n = side * side, c = side / 2;
    const long long base = (long long)k * n;
    const float *P = pred + base * cpad;
    const double *R0 = rho0 + base;
    double *RO = rho_out + base;
    double *UX = u_out + base, *UY = u_out + ntot + base, *UZ = u_out + 2 * ntot + base;
    // the eight matrices (a b; c d) acting on (X, Y) relative to the centre
    const int ma[8] = {1, -1, 1, -1, 0, 0, 0, 0}, mb[8] = {0, 0, 0, 0, 1, -1, 1, -1};
    const int mc[8] = {0, 0, 0, 0, 1, 1, -1, -1}, md[8] = {1, 1, -1, -1, 0, 0, 0, 0};
    const int ng = sym ? 8 : 1;

    double acc[3] = {0.0, 0.0, 0.0};  // predicted mass, cold mass, bad count
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        const int X = s % side - c, Y = s / side - c;
        double r = 0.0, ux = 0.0, uy = 0.0;
        for (int g = 0; g < ng; g++) {
            int xs = c + ma[g] * X + mb[g] * Y, ys = c + mc[g] * X + md[g] * Y;
            xs = ((xs % side) + side) % side;
            ys = ((ys % side) + side) % side;
            const int q = ys * side + xs;
            const float *pq = P + (long long)q * cpad;
            const double p0 = pq[0];
            if (!isfinite(p0)) acc[2] += 1.0;
            r += R0[q] + s_rho * p0;
            if (with_u) {
                const double vx = pq[1], vy = pq[2];
                if (!(isfinite(vx) && isfinite(vy))) acc[2] += 1.0;
                ux += s_u * (ma[g] * vx + mc[g] * vy);
                uy += s_u * (mb[g] * vx + md[g] * vy);
            }
        }
        const double inv = 1.0 / ng;
        RO[s] = r * inv;
        UX[s] = ux * inv;
        UY[s] = uy * inv;
        acc[0] += r * inv;
        acc[1] += R0[s];
    }
    block_sum<3>(acc);
    const bool bad = acc[2] != 0.0;
    const double shift = (acc[1] - acc[0]) / n;
    double mom[3] = {0.0, 0.0, 0.0};  // mass, x momentum, y momentum
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        double r = bad ? R0[s] : fmin(fmax(RO[s] + shift, rho_lo), rho_hi);
        double ux = bad ? 0.0 : UX[s], uy = bad ? 0.0 : UY[s];
        RO[s] = r;
        UX[s] = ux;
        UY[s] = uy;
        mom[0] += r;
        mom[1] += r * ux;
        mom[2] += r * uy;
    }
    block_sum<3>(mom);
    const double mx = mom[1] / mom[0], my = mom[2] / mom[0];
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        UX[s] -= mx;
        UY[s] -= my;
        UZ[s] = 0.0;
    }
}

} // namespace lbmwarm
