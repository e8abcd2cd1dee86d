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
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Four FP32 values rounded to bf16 (round to nearest even, the hardware
// conversion) and packed as one MFMA operand.
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d)
{
    const unsigned lo = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2_t));
    const unsigned hi = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){c, d}, bf16x2_t));
    bf16x4 r;
    r[0] = short(lo & 0xFFFFu);
    r[1] = short(lo >> 16);
    r[2] = short(hi & 0xFFFFu);
    r[3] = short(hi >> 16);
    return r;
}

struct ConvShape {
    int nb, h, w;     // images, rows, columns (nb h w < 2^31, checked by the host)
    int cin, cout;    // padded channel counts (multiples of 16)
    int cout_real;    // channels beyond this are written as zero
};

// Pixel p = (b h + y) w + x and its periodic neighbours.
struct Pix {
    int b, y, x;
};
__device__ __forceinline__ Pix pix_of(const ConvShape &s, int p)
{
    const int r = p / s.w;
    return Pix{r / s.h, r % s.h, p - r * s.w};
}
__device__ __forceinline__ int pix_at(const ConvShape &s, Pix q, int dy, int dx)
{
    int ys = q.y + dy, xs = q.x + dx;
    ys = ys < 0 ? ys + s.h : (ys >= s.h ? ys - s.h : ys);
    xs = xs < 0 ? xs + s.w : (xs >= s.w ? xs - s.w : xs);
    return (q.b * s.h + ys) * s.w + xs;
}

constexpr int CONV_MT = 4;  // 16-pixel tiles per wave in the forward / data-gradient kernels

// B operands of all (tap, n-tile, k-tile) MFMA blocks, bf16, in the layout a
// lane reads them: lane l holds B[k = 4 (l / 16) + j][n = l % 16], j = 0..3.
// transpose = false: B[k = ci][n = co] = W[tap][co][ci] (forward);
// transpose = true:  B[k = co][n = ci] = W[tap][co][ci] (data gradient).
__device__ __forceinline__ void stage_weights(const ConvShape &s, const float *__restrict__ wt, bool transpose,
                                              bf16x4 *__restrict__ lds)
{
    const int kdim = transpose ? s.cout : s.cin, ndim = transpose ? s.cin : s.cout;
    const int kt_n = kdim / 16, nt_n = ndim / 16;
    const int total = 9 * nt_n * kt_n * 64;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int l = e & 63, blk = e >> 6;
        const int kt = blk % kt_n, nt = (blk / kt_n) % nt_n, tap = blk / (kt_n * nt_n);
        const int n = nt * 16 + (l & 15), k = kt * 16 + 4 * (l >> 4);
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int co = transpose ? k + j : n, ci = transpose ? n : k + j;
            v[j] = wt[((long long)tap * s.cout + co) * s.cin + ci];
        }
        lds[e] = pack4(v[0], v[1], v[2], v[3]);
    }
}

// out[p][co] = bias[co] + sum_{tap, ci} W[tap][co][ci] act(in[p + off(tap)][ci]),
// act = relu when relu_in, else identity.  A workgroup stages the weights in
// LDS as bf16 once; each wave computes CONV_MT tiles of 16 pixels x all cout
// (A[m = pixel][k = ci] from the input, B from LDS).
// Requires nb * h * w % 16 == 0 and cout <= 32.
__global__ __launch_bounds__(NET_THREADS) void conv_fwd_kernel(ConvShape s, const float *__restrict__ in,
                                                               int relu_in, const float *__restrict__ wt,
                                                               const float *__restrict__ bias,
                                                               float *__restrict__ out)
{
    __shared__ bf16x4 wl[9 * 2 * 2 * 64];
    stage_weights(s, wt, false, wl);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int npix = s.nb * s.h * s.w;
    const int m0 = (blockIdx.x * 4 + wave) * 16 * CONV_MT;
    if (m0 >= npix) return;
    const int r = lane & 15, g = lane >> 4;  // row within the 16 x 16 tile, k group
    const int nt_n = s.cout / 16, kt_n = s.cin / 16;
    const int mt_n = min(CONV_MT, (npix - m0) / 16);
    Pix px[CONV_MT];
#pragma unroll
    for (int t = 0; t < CONV_MT; t++) px[t] = pix_of(s, min(m0 + 16 * t + r, npix - 1));
    f32x4 acc[CONV_MT][2];
#pragma unroll
    for (int t = 0; t < CONV_MT; t++) acc[t][0] = acc[t][1] = (f32x4){0, 0, 0, 0};
    for (int tap = 0; tap < 9; tap++) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        int q[CONV_MT];
#pragma unroll
        for (int t = 0; t < CONV_MT; t++) q[t] = pix_at(s, px[t], dy, dx);
        for (int kt = 0; kt < kt_n; kt++) {
            const bf16x4 B0 = wl[((tap * nt_n + 0) * kt_n + kt) * 64 + lane];
            const bf16x4 B1 = nt_n > 1 ? wl[((tap * nt_n + 1) * kt_n + kt) * 64 + lane] : B0;
#pragma unroll
            for (int t = 0; t < CONV_MT; t++) {
                if (t >= mt_n) break;
                const float4 a4 = *reinterpret_cast<const float4 *>(in + (long long)q[t] * s.cin + kt * 16 + 4 * g);
                float a0 = a4.x, a1 = a4.y, a2 = a4.z, a3 = a4.w;
                if (relu_in) {
                    a0 = fmaxf(a0, 0.f); a1 = fmaxf(a1, 0.f); a2 = fmaxf(a2, 0.f); a3 = fmaxf(a3, 0.f);
                }
                const bf16x4 A = pack4(a0, a1, a2, a3);
                acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B0, acc[t][0], 0, 0, 0);
                if (nt_n > 1) acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B1, acc[t][1], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < CONV_MT; t++) {
        if (t >= mt_n) break;
        for (int nt = 0; nt < nt_n; nt++) {
            const int co = nt * 16 + r;
            const float bv = co < s.cout_real ? bias[co] : 0.f;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const long long p = m0 + 16 * t + 4 * g + j;
                out[p * s.cout + co] = co < s.cout_real ? acc[t][nt][j] + bv : 0.f;
            }
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
    __shared__ bf16x4 wl[9 * 2 * 2 * 64];
    stage_weights(s, wt, true, wl);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int npix = s.nb * s.h * s.w;
    const int m0 = (blockIdx.x * 4 + wave) * 16 * CONV_MT;
    if (m0 >= npix) return;
    const int r = lane & 15, g = lane >> 4;
    const int nt_n = s.cin / 16, kt_n = s.cout / 16;  // output: cin channels; sum over cout
    const int mt_n = min(CONV_MT, (npix - m0) / 16);
    Pix px[CONV_MT];
#pragma unroll
    for (int t = 0; t < CONV_MT; t++) px[t] = pix_of(s, min(m0 + 16 * t + r, npix - 1));
    f32x4 acc[CONV_MT][2];
#pragma unroll
    for (int t = 0; t < CONV_MT; t++) acc[t][0] = acc[t][1] = (f32x4){0, 0, 0, 0};
    for (int tap = 0; tap < 9; tap++) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        int q[CONV_MT];
#pragma unroll
        for (int t = 0; t < CONV_MT; t++) q[t] = pix_at(s, px[t], -dy, -dx);
        for (int kt = 0; kt < kt_n; kt++) {
            const bf16x4 B0 = wl[((tap * nt_n + 0) * kt_n + kt) * 64 + lane];
            const bf16x4 B1 = nt_n > 1 ? wl[((tap * nt_n + 1) * kt_n + kt) * 64 + lane] : B0;
#pragma unroll
            for (int t = 0; t < CONV_MT; t++) {
                if (t >= mt_n) break;
                const float4 a4 =
                    *reinterpret_cast<const float4 *>(dout + (long long)q[t] * s.cout + kt * 16 + 4 * g);
                const bf16x4 A = pack4(a4.x, a4.y, a4.z, a4.w);
                acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B0, acc[t][0], 0, 0, 0);
                if (nt_n > 1) acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B1, acc[t][1], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < CONV_MT; t++) {
        if (t >= mt_n) break;
        for (int nt = 0; nt < nt_n; nt++) {
            const int ci = nt * 16 + r;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const long long p = m0 + 16 * t + 4 * g + j;
                float v = acc[t][nt][j];
                if (zin && !(zin[p * s.cin + ci] > 0.f)) v = 0.f;
                din[p * s.cin + ci] = v;
            }
        }
    }
}

// Partial weight gradients of one workgroup's pixel chunk:
// part[wg][tap][co][ci] = sum_{p in chunk} dout[p][co] act(in[p + off(tap)][ci]),
// followed by the bias gradient part[wg][9 cout cin + co] = sum_{p in chunk}
// dout[p][co] (FP32, from the unrounded values).
// The contraction runs over pixels, which are the strided index of the NHWC
// tensors, so each block of 64 pixels is first staged in LDS as bf16 with
// the pixel index contiguous (dout as [co][px], the shifted inputs of all
// nine taps as [tap][ci][px]); a wave then owns one (co-tile, ci-tile) block
// and a group of taps and reads both MFMA operands from LDS.
constexpr int BW_PX = 64;  // pixels per staged block
__global__ __launch_bounds__(NET_THREADS) void conv_bwd_weight_kernel(ConvShape s,
                                                                      const float *__restrict__ dout,
                                                                      const float *__restrict__ in,
                                                                      int relu_in, int chunk,
                                                                      float *__restrict__ part)
{
    __shared__ __bf16 sa[32 * BW_PX];      // [co][px]
    __shared__ __bf16 sb[9 * 32 * BW_PX];  // [tap][ci][px]
    __shared__ float sbias[32 * BW_PX];    // per-thread bias partials [co][pi]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int npix = s.nb * s.h * s.w;
    const int p0 = blockIdx.x * chunk;
    const int p1 = min(p0 + chunk, npix);
    const int r = lane & 15, g = lane >> 4;
    const int cot = s.cout / 16, cit = s.cin / 16;
    const int nblk = cot * cit;              // 1, 2 or 4 blocks
    const int groups = 4 / nblk;             // tap groups per block
    const int blk = wave % nblk, grp = wave / nblk;
    const int ct = blk / cit, it = blk % cit;
    const int tap0 = (9 * grp) / groups, tap1 = (9 * (grp + 1)) / groups;
    // staging role of this thread: pixel pi of the block, channels 8 cg .. 8 cg + 7
    const int pi = threadIdx.x % BW_PX, cg = threadIdx.x / BW_PX;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; t++) acc[t] = (f32x4){0, 0, 0, 0};
    float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int pb = p0; pb < p1; pb += BW_PX) {
        const int p = pb + pi;
        const bool ok = p < p1;
        const Pix px = pix_of(s, ok ? p : p0);
        if (8 * cg < s.cout) {
            float v[8];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                float4 f = ok ? *reinterpret_cast<const float4 *>(dout + (long long)p * s.cout + 8 * cg + 4 * h)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
                v[4 * h] = f.x; v[4 * h + 1] = f.y; v[4 * h + 2] = f.z; v[4 * h + 3] = f.w;
            }
#pragma unroll
            for (int c = 0; c < 8; c++) {
                sa[(8 * cg + c) * BW_PX + pi] = (__bf16)v[c];
                bsum[c] += v[c];
            }
        }
        if (8 * cg < s.cin) {
            for (int tap = 0; tap < 9; tap++) {
                const int q = pix_at(s, px, tap / 3 - 1, tap % 3 - 1);
                float v[8];
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    float4 f = ok ? *reinterpret_cast<const float4 *>(in + (long long)q * s.cin + 8 * cg + 4 * h)
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
                    v[4 * h] = f.x; v[4 * h + 1] = f.y; v[4 * h + 2] = f.z; v[4 * h + 3] = f.w;
                }
#pragma unroll
                for (int c = 0; c < 8; c++)
                    sb[(tap * 32 + 8 * cg + c) * BW_PX + pi] = (__bf16)(relu_in ? fmaxf(v[c], 0.f) : v[c]);
            }
        }
        __syncthreads();
        // A[m = co][k = pixel], B[k = pixel][n = ci]: lane holds k = 4 g .. 4 g + 3
#pragma unroll
        for (int ks = 0; ks < BW_PX / 16; ks++) {
            const bf16x4 A = *reinterpret_cast<const bf16x4 *>(sa + (ct * 16 + r) * BW_PX + 16 * ks + 4 * g);
#pragma unroll
            for (int tap = 0; tap < 9; tap++) {
                if (tap < tap0 || tap >= tap1) continue;
                const bf16x4 B =
                    *reinterpret_cast<const bf16x4 *>(sb + (tap * 32 + it * 16 + r) * BW_PX + 16 * ks + 4 * g);
                acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[tap], 0, 0, 0);
            }
        }
        __syncthreads();  // the staging buffers are refilled next
    }
    // D[m = co][n = ci]: lane holds rows 4g..4g+3 of column r
    float *mypart = part + (long long)blockIdx.x * (9 * s.cout * s.cin + s.cout);
    // bias partials: the 64 staging threads of a channel group, in order
    if (8 * cg < s.cout) {
#pragma unroll
        for (int c = 0; c < 8; c++) sbias[(8 * cg + c) * BW_PX + pi] = bsum[c];
    }
    __syncthreads();
    if (threadIdx.x < s.cout) {
        float b = 0.f;
        for (int k = 0; k < BW_PX; k++) b += sbias[threadIdx.x * BW_PX + k];
        mypart[9 * s.cout * s.cin + threadIdx.x] = b;
    }
#pragma unroll
    for (int tap = 0; tap < 9; tap++) {
        if (tap < tap0 || tap >= tap1) continue;
#pragma unroll
        for (int j = 0; j < 4; j++)
            mypart[((long long)tap * s.cout + ct * 16 + 4 * g + j) * s.cin + it * 16 + r] = acc[tap][j];
    }
}

// Sum nparts rows of length len: v_i = sum_k part[k][i], in a fixed order
// (four consecutive ranges of k summed by four waves, then combined in
// order), written to out_a[i] for i < na and to out_b[i - na] after that.
// 64 columns per workgroup of 256 threads.
__global__ __launch_bounds__(256) void sum_parts_kernel(int nparts, int len, int na,
                                                        const float *__restrict__ part,
                                                        float *__restrict__ out_a, float *__restrict__ out_b)
{
    __shared__ float sh[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int k0 = (nparts * wave) / 4, k1 = (nparts * (wave + 1)) / 4;
    float a = 0.f;
    if (i < len)
        for (int k = k0; k < k1; k++) a += part[(long long)k * len + i];
    sh[wave][lane] = a;
    __syncthreads();
    if (wave == 0 && i < len) {
        const float v = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
        if (i < na)
            out_a[i] = v;
        else
            out_b[i - na] = v;
    }
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
