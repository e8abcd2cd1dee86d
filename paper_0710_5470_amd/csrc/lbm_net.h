// lbm_net.h -- kernels of the warm-start network: 3x3 periodic convolutions
// (forward, backward-data, backward-weight) as implicit GEMMs on bf16 MFMA
// (v_mfma_f32_16x16x16_bf16) with FP32 accumulation, plus the loss and the
// Adam update.
//
// Tensors are FP32 in memory, NHWC with the channel count padded to a
// multiple of 16 (the MFMA K / N tile); operands are rounded to bf16 (round
// to nearest even) as they are fed to the matrix cores.  Convolutions wrap
// periodically in x and y, like the lattice the network predicts.
// Weights are stored [tap][cout][cin] with tap = 3 (dy + 1) + (dx + 1), so
// out[p] = b + sum_tap W[tap] . in[p + (dy, dx)].
#pragma once

#include <hip/hip_runtime.h>

namespace lbmnet {

constexpr int NET_THREADS = 256;  // 4 waves

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f)
{
    unsigned u = __builtin_bit_cast(unsigned, f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return short(u >> 16);
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d)
{
    bf16x4 r;
    r[0] = to_bf16(a);
    r[1] = to_bf16(b);
    r[2] = to_bf16(c);
    r[3] = to_bf16(d);
    return r;
}

struct ConvShape {
    int nb, h, w;     // images, rows, columns
    int cin, cout;    // padded channel counts (multiples of 16)
    int cout_real;    // channels beyond this are written as zero
};

__device__ __forceinline__ long long pix_shift(const ConvShape &s, long long p, int dy, int dx)
{
    const int x = int(p % s.w);
    const long long r = p / s.w;
    const int y = int(r % s.h);
    const long long b = r / s.h;
    int ys = y + dy, xs = x + dx;
    ys = ys < 0 ? ys + s.h : (ys >= s.h ? ys - s.h : ys);
    xs = xs < 0 ? xs + s.w : (xs >= s.w ? xs - s.w : xs);
    return (b * s.h + ys) * s.w + xs;
}

// out[p][co] = bias[co] + sum_{tap, ci} W[tap][co][ci] act(in[p + off(tap)][ci]),
// act = relu when relu_in, else identity.  One wave: 16 pixels x all cout.
// Requires nb * h * w % 16 == 0 and cout <= 32.
__global__ __launch_bounds__(NET_THREADS) void conv_fwd_kernel(ConvShape s, const float *__restrict__ in,
                                                               int relu_in, const float *__restrict__ wt,
                                                               const float *__restrict__ bias,
                                                               float *__restrict__ out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long npix = (long long)s.nb * s.h * s.w;
    const long long m0 = ((long long)blockIdx.x * 4 + wave) * 16;
    if (m0 >= npix) return;
    const int r = lane & 15, g = lane >> 4;  // row within the 16 x 16 tile, k group
    const int ntile = s.cout / 16;
    f32x4 acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int tap = 0; tap < 9; tap++) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const long long q = pix_shift(s, m0 + r, dy, dx);
        for (int kk = 0; kk < s.cin; kk += 16) {
            const float4 a4 = *reinterpret_cast<const float4 *>(in + q * s.cin + kk + 4 * g);
            float a0 = a4.x, a1 = a4.y, a2 = a4.z, a3 = a4.w;
            if (relu_in) {
                a0 = fmaxf(a0, 0.f); a1 = fmaxf(a1, 0.f); a2 = fmaxf(a2, 0.f); a3 = fmaxf(a3, 0.f);
            }
            const bf16x4 A = pack4(a0, a1, a2, a3);
            for (int nt = 0; nt < ntile; nt++) {
                const int co = nt * 16 + r;
                const float4 b4 =
                    *reinterpret_cast<const float4 *>(wt + ((long long)tap * s.cout + co) * s.cin + kk + 4 * g);
                const bf16x4 B = pack4(b4.x, b4.y, b4.z, b4.w);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[nt], 0, 0, 0);
            }
        }
    }
    for (int nt = 0; nt < ntile; nt++) {
        const int co = nt * 16 + r;
        for (int j = 0; j < 4; j++) {
            const long long p = m0 + 4 * g + j;
            out[p * s.cout + co] = co < s.cout_real ? acc[nt][j] + bias[co] : 0.f;
        }
    }
}

// din[q][ci] = mask(q, ci) * sum_{tap, co} W[tap][co][ci] dout[q - off(tap)][co],
// mask = (zin[q][ci] > 0) when zin is given (relu of the previous layer).
// s describes the forward convolution (cin = its input, cout = its output).
__global__ __launch_bounds__(NET_THREADS) void conv_bwd_data_kernel(ConvShape s,
                                                                    const float *__restrict__ dout,
                                                                    const float *__restrict__ wt,
                                                                    const float *__restrict__ zin,
                                                                    float *__restrict__ din)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long npix = (long long)s.nb * s.h * s.w;
    const long long m0 = ((long long)blockIdx.x * 4 + wave) * 16;
    if (m0 >= npix) return;
    const int r = lane & 15, g = lane >> 4;
    const int ntile = s.cin / 16;  // output of this kernel: cin channels
    f32x4 acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int tap = 0; tap < 9; tap++) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const long long q = pix_shift(s, m0 + r, -dy, -dx);
        for (int kk = 0; kk < s.cout; kk += 16) {
            const float4 a4 = *reinterpret_cast<const float4 *>(dout + q * s.cout + kk + 4 * g);
            const bf16x4 A = pack4(a4.x, a4.y, a4.z, a4.w);
            for (int nt = 0; nt < ntile; nt++) {
                const int ci = nt * 16 + r;
                const float *wp = wt + ((long long)tap * s.cout + kk + 4 * g) * s.cin + ci;
                const bf16x4 B = pack4(wp[0], wp[s.cin], wp[2 * s.cin], wp[3 * s.cin]);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[nt], 0, 0, 0);
            }
        }
    }
    for (int nt = 0; nt < ntile; nt++) {
        const int ci = nt * 16 + r;
        for (int j = 0; j < 4; j++) {
            const long long p = m0 + 4 * g + j;
            float v = acc[nt][j];
            if (zin && !(zin[p * s.cin + ci] > 0.f)) v = 0.f;
            din[p * s.cin + ci] = v;
        }
    }
}

// Partial weight gradients of one workgroup's pixel chunk:
// part[wg][tap][co][ci] = sum_{p in chunk} dout[p][co] act(in[p + off(tap)][ci]).
// Each wave owns 9 of the 36 (tap, co-tile, ci-tile) blocks (cin, cout <= 32).
__global__ __launch_bounds__(NET_THREADS) void conv_bwd_weight_kernel(ConvShape s,
                                                                      const float *__restrict__ dout,
                                                                      const float *__restrict__ in,
                                                                      int relu_in, int chunk,
                                                                      float *__restrict__ part)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long npix = (long long)s.nb * s.h * s.w;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = p0 + chunk < npix ? p0 + chunk : npix;
    const int r = lane & 15, g = lane >> 4;
    const int cot = s.cout / 16, cit = s.cin / 16;
    const int nblk = 9 * cot * cit;
    float *mypart = part + (long long)blockIdx.x * 9 * s.cout * s.cin;
    for (int blk = wave; blk < nblk; blk += 4) {
        const int tap = blk / (cot * cit), ct = (blk / cit) % cot, it = blk % cit;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        f32x4 acc = {0, 0, 0, 0};
        for (long long pk = p0; pk < p1; pk += 16) {
            // A[m = co][k = pixel], B[k = pixel][n = ci]
            float a[4], b[4];
            for (int j = 0; j < 4; j++) {
                const long long p = pk + 4 * g + j;
                const bool ok = p < p1;
                a[j] = ok ? dout[p * s.cout + ct * 16 + r] : 0.f;
                float v = ok ? in[pix_shift(s, ok ? p : 0, dy, dx) * s.cin + it * 16 + r] : 0.f;
                b[j] = relu_in ? fmaxf(v, 0.f) : v;
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pack4(a[0], a[1], a[2], a[3]),
                                                            pack4(b[0], b[1], b[2], b[3]), acc, 0, 0, 0);
        }
        // D[m = co][n = ci]: lane holds rows 4g..4g+3 of column r
        for (int j = 0; j < 4; j++)
            mypart[((long long)tap * s.cout + ct * 16 + 4 * g + j) * s.cin + it * 16 + r] = acc[j];
    }
}

// Sum nparts rows of length len in index order: out[i] = sum_k part[k][i].
__global__ void sum_parts_kernel(int nparts, int len, const float *__restrict__ part, float *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    float a = 0.f;
    for (int k = 0; k < nparts; k++) a += part[(long long)k * len + i];
    out[i] = a;
}

// dbias[co] = sum_p dout[p][co]: one workgroup per channel, fixed tree.
__global__ __launch_bounds__(NET_THREADS) void bias_grad_kernel(long long npix, int cout,
                                                                const float *__restrict__ dout,
                                                                float *__restrict__ dbias)
{
    __shared__ float sh[NET_THREADS];
    const int co = blockIdx.x;
    float a = 0.f;
    for (long long p = threadIdx.x; p < npix; p += NET_THREADS) a += dout[p * cout + co];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = NET_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) dbias[co] = sh[0];
}

// Mean squared error over the first `creal` of `c` channels:
// grad = 2 (pred - target) / count, per-workgroup partial sums of squares.
__global__ __launch_bounds__(NET_THREADS) void mse_kernel(long long npix, int c, int creal,
                                                          const float *__restrict__ pred,
                                                          const float *__restrict__ target,
                                                          float *__restrict__ grad,
                                                          double *__restrict__ part)
{
    __shared__ double sh[NET_THREADS];
    const double inv = 1.0 / (double(npix) * creal);
    double a = 0.0;
    const long long n = npix * c;
    for (long long i = (long long)blockIdx.x * NET_THREADS + threadIdx.x; i < n;
         i += (long long)gridDim.x * NET_THREADS) {
        const int ch = int(i % c);
        float d = ch < creal ? pred[i] - target[i] : 0.f;
        grad[i] = float(2.0 * inv) * d;
        a += double(d) * double(d);
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = NET_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] * inv;
}

// Adam (Kingma & Ba, 2015) with bias correction, in place.
__global__ void adam_kernel(int n, float *__restrict__ p, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

} // namespace lbmnet
