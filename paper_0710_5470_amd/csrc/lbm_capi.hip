// lbm_capi.hip -- host side of the C ABI declared in include/lbm.h.
//
// Holds the context, turns the physical parameters into kernel
// coefficients, carves the caller's workspace, dispatches the templated
// kernels and runs the FP64 reductions.  Also the host Maxwell solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>

#include "lbm.h"  // include/, on the include path
#include "lbm_aux.h"
#include "lbm_step.h"

using namespace lbm;

// the D3Q19 step kernels come from lbm_step3d.hip
namespace lbm {
#define LBM_STEP3D_EXTERN(SCH, S, R, TX, TY) \
    extern template __global__ void step_kernel<D3Q19, SCH, S, R, TX, TY>(StepArgs<R>);
LBM_STEP3D_INSTANCES(LBM_STEP3D_EXTERN)
#undef LBM_STEP3D_EXTERN
} // namespace lbm

namespace {

constexpr int RED_BLOCKS = 1024;
constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct TileShape {
    int tx, ty;
};
// D2Q9 marches along y with a row of tx sites; D3Q19 marches along z.
constexpr TileShape TILES_2D[] = {{64, 1}, {128, 1}, {256, 1}};
constexpr TileShape TILES_3D[] = {{64, 4}, {32, 8}, {64, 8}, {32, 16}, {128, 4}};
constexpr int NT2 = sizeof(TILES_2D) / sizeof(TILES_2D[0]);
constexpr int NT3 = sizeof(TILES_3D) / sizeof(TILES_3D[0]);

struct Layout {
    size_t pops;      // bytes of one population buffer
    size_t off_a, off_b, off_rho, off_vel, off_prev, off_part, off_res, total;
};

bool valid_params(const lbm_params *p)
{
    if (!p) return false;
    if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q19) return false;
    if (p->scheme != LBM_SCHEME_EQ && p->scheme != LBM_SCHEME_FORCE) return false;
    if (p->storage != LBM_STORE_F64 && p->storage != LBM_STORE_F32_SHIFTED) return false;
    if (p->shift_mode != LBM_SHIFT_REST_EQ && p->shift_mode != LBM_SHIFT_WEIGHTS) return false;
    if (p->compute != LBM_COMPUTE_NATIVE && p->compute != LBM_COMPUTE_F64) return false;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
    if (p->lattice == LBM_D2Q9 && p->nz != 1) return false;
    // a population buffer is addressed with 32-bit byte offsets
    double es = p->storage == LBM_STORE_F64 ? 8.0 : 4.0;
    if ((double)p->nx * p->ny * p->nz * es * p->lattice >= 4294967296.0) return false;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return false;
    if (!(p->T > 0.0) || !std::isfinite(p->T)) return false;
    if (!(p->a >= 0.0) || !(p->b >= 0.0) || !(p->kappa >= 0.0)) return false;
    if (!std::isfinite(p->a) || !std::isfinite(p->b) || !std::isfinite(p->kappa)) return false;
    if (p->lattice == LBM_D3Q19 &&
        (!std::isnan(p->wp_diag) || !std::isnan(p->wt_diag) || !std::isnan(p->wxx_diag)))
        return false;
    int nt = p->lattice == LBM_D2Q9 ? NT2 : NT3;
    if (p->tile >= nt) return false;
    return true;
}

Layout layout(const lbm_params *p)
{
    Layout L{};
    size_t n = (size_t)p->nx * p->ny * p->nz;
    size_t es = p->storage == LBM_STORE_F64 ? 8 : 4;
    L.pops = align_up(n * p->lattice * es);
    size_t o = 0;
    L.off_a = o; o += L.pops;
    L.off_b = o; o += L.pops;
    L.off_rho = o; o += align_up(n * 8);
    L.off_vel = o; o += align_up(3 * n * 8);
    L.off_prev = o; o += align_up(3 * n * 8);
    L.off_part = o; o += align_up((size_t)RED_BLOCKS * 20 * 8);
    L.off_res = o; o += align_up(32 * 8);
    L.total = o;
    return L;
}

} // namespace

struct lbm_ctx {
    lbm_params p;
    Layout lay;
    char *ws;
    hipStream_t stream;
    int cur;               // 0: state in buffer A, 1: in buffer B
    long long steps;
    int tile, cp;
    Coefs<double> cd;      // FP64 coefficients (init, exchange, FP64 steps)
    Coefs<float> cf;       // FP32 coefficients
    int nx, ny, np;        // kernel geometry
    long long n;
    bool prev_valid;       // observation field "prev" holds the previous step
};

namespace {

void *buf_cur(lbm_ctx *c) { return c->ws + (c->cur ? c->lay.off_b : c->lay.off_a); }
void *buf_nxt(lbm_ctx *c) { return c->ws + (c->cur ? c->lay.off_a : c->lay.off_b); }
double *ws_d(lbm_ctx *c, size_t off) { return reinterpret_cast<double *>(c->ws + off); }

double pick(double v, double dflt) { return std::isnan(v) ? dflt : v; }

// Coefficients of Eqs. (xderiv), (laplace), (laplacian3d), the equilibrium
// weights (summary / Eq. (3dres)) and the force stencil.
Coefs<double> make_coefs(const lbm_params *p)
{
    Coefs<double> c{};
    bool d3 = p->lattice == LBM_D3Q19;
    double B = pick(p->B, 1.0 / 12.0), D = pick(p->D, 1.0 / 6.0), F = pick(p->F, 1.0 / 12.0);
    if (!d3) {
        c.A = (1.0 - 4.0 * B) / 2.0;       // 2A + 4B = 1
        c.C = 1.0 - 2.0 * D;               // C + 2D = 1
        c.Ef = (1.0 - 4.0 * F) / 2.0;
        c.w_ax = 1.0 / 3.0;
        c.w_off = 1.0 / 12.0;
        double wp = pick(p->wp_diag, 1.0 / 12.0), wt = pick(p->wt_diag, 1.0 / 12.0);
        double wxx = pick(p->wxx_diag, -1.0 / 24.0);
        c.wp_off = wp;
        c.wp_ax = 0.5 - 2.0 * wp;          // 2 w_1-4 + 4 w_5-8 = 1
        c.wt_off = wt;
        c.wt_ax = 0.5 - 2.0 * wt;
        c.wm_para = 0.25 - 2.0 * wxx;      // 2 w^xx_1-2 + 4 w^xx_5-8 = 1/2
        c.wm_perp = -0.25 - 2.0 * wxx;     // 2 w^yy_1-2 + 4 w^yy_5-8 = -1/2
        c.wm_in = wxx;
        c.wm_out = 0.0;
    } else {
        c.A = (1.0 - 8.0 * B) / 2.0;       // 2A + 8B = 1
        c.C = 1.0 - 4.0 * D;               // C + 4D = 1
        c.Ef = (1.0 - 8.0 * F) / 2.0;
        c.w_ax = 1.0 / 6.0;
        c.w_off = 1.0 / 12.0;
        c.wp_ax = c.wt_ax = 1.0 / 6.0;
        c.wp_off = c.wt_off = 1.0 / 12.0;
        c.wm_para = 5.0 / 12.0;
        c.wm_perp = -1.0 / 3.0;
        c.wm_in = -1.0 / 24.0;
        c.wm_out = 1.0 / 12.0;
    }
    c.B = B;
    c.D = D;
    c.Ff = F;
    c.a = p->a;
    c.b = p->b;
    c.T = p->T;
    c.kappa = p->kappa;
    c.omega = 1.0 / p->tau;
    c.ow_ax = c.omega * c.w_ax;
    c.ow_off = c.omega * c.w_off;
    c.nu = (p->tau - 0.5) / 3.0;
    c.lambda_on = p->galilean_lambda ? 1 : 0;
    c.wp_ax_d = c.wp_ax;
    c.wp_off_d = c.wp_off;
    return c;
}

// Per-direction FP32 shift (see LBM_SHIFT_*), symmetric under e -> -e.
void make_shift(const lbm_params *p, Coefs<double> &c, double rho0)
{
    for (int i = 0; i < 19; i++) c.shift[i] = 0.0;
    c.shift_sum = 0.0;
    if (p->storage == LBM_STORE_F64) return;
    int q = p->lattice;
    bool d3 = q == LBM_D3Q19;
    double sum = 0.0;
    for (int i = 1; i < q; i++) {
        int nz = d3 ? nnz<D3Q19>(i) : nnz<D2Q9>(i);
        if (p->shift_mode == LBM_SHIFT_WEIGHTS)
            c.shift[i] = (nz == 1 ? (d3 ? 1.0 / 18.0 : 1.0 / 9.0) : 1.0 / 36.0) * rho0;
        else {
            double p0 = rho0 * p->T / (1.0 - p->b * rho0) - p->a * rho0 * rho0;
            c.shift[i] = (nz == 1 ? c.wp_ax : c.wp_off) * p0;
        }
        c.shift[i] = double(float(c.shift[i]));  // the FP32 kernels see these exact values
        sum += c.shift[i];
    }
    c.shift[0] = double(float(rho0 - sum));
    c.shift_sum = sum + c.shift[0];
}

// FP32 weights (a, o) of the axis and off-axis classes with 2 a + m o = t
// holding exactly (m: off-axis velocities with a nonzero component along a
// given axis, 4 in D2Q9 and 8 in D3Q19).  One of the two is rounded, the
// other solved for; the first choice whose identity holds exactly is kept
// (both are exact in FP64, which holds the products of FP32 values
// exactly).  Rounding both independently would break the first-moment
// identity sum_i w_i e_ia e_ib = delta_ab by ~1e-8: the collision would then
// create momentum omega (2 a + m o - 1) j every step, a bias that moves the
// FP32 state away from the conserved dynamics.
void exact_pair(double a, double o, float t, int m, float &fa, float &fo)
{
    fa = float(a);
    fo = float((double(t) - 2.0 * double(fa)) / m);
    if (2.0 * double(fa) + m * double(fo) == double(t)) return;
    fo = float(o);
    fa = float((double(t) - m * double(fo)) / 2.0);
    if (2.0 * double(fa) + m * double(fo) == double(t)) return;
    fa = float(a);  // no exact pair: plain rounding
    fo = float(o);
}

Coefs<float> to_float(const Coefs<double> &d, int lattice)
{
    Coefs<float> f{};
    const int m = lattice == LBM_D3Q19 ? 8 : 4;
    f.A = float(d.A); f.B = float(d.B); f.C = float(d.C); f.D = float(d.D);
    f.Ef = float(d.Ef); f.Ff = float(d.Ff);
    f.omega = float(d.omega);
    exact_pair(d.w_ax, d.w_off, 1.0f, m, f.w_ax, f.w_off);
    exact_pair(d.ow_ax, d.ow_off, f.omega, m, f.ow_ax, f.ow_off);
    f.wp_ax = float(d.wp_ax); f.wp_off = float(d.wp_off);
    f.wt_ax = float(d.wt_ax); f.wt_off = float(d.wt_off);
    f.wm_para = float(d.wm_para); f.wm_perp = float(d.wm_perp);
    f.wm_in = float(d.wm_in); f.wm_out = float(d.wm_out);
    f.kappa = float(d.kappa);
    f.lambda_on = d.lambda_on;
    f.a = d.a; f.b = d.b; f.T = d.T; f.nu = d.nu;
    f.wp_ax_d = d.wp_ax_d; f.wp_off_d = d.wp_off_d;
    for (int i = 0; i < 19; i++) f.shift[i] = d.shift[i];
    f.shift_sum = d.shift_sum;
    return f;
}

TileShape tile_shape(int lattice, int t)
{
    return lattice == LBM_D2Q9 ? TILES_2D[t] : TILES_3D[t];
}

int default_tile(const lbm_params *p)
{
    if (p->lattice == LBM_D2Q9) return p->nx >= 256 ? 2 : (p->nx >= 128 ? 1 : 0);
    return 1;  // 32 x 8
}

void grid_of(const lbm_ctx *c, int tile, int cp, int &tx_n, int &ty_n, int &chunks)
{
    TileShape t = tile_shape(c->p.lattice, tile);
    tx_n = (c->nx + t.tx - 1) / t.tx;
    ty_n = (c->ny + t.ty - 1) / t.ty;
    chunks = (c->np + cp - 1) / cp;
}

int default_planes(const lbm_ctx *c, int tile)
{
    int tx_n, ty_n, ch;
    grid_of(c, tile, 1, tx_n, ty_n, ch);
    long long tiles = (long long)tx_n * ty_n;
    // aim for about 4096 workgroups, marching at least 8 planes where the
    // lattice allows (fewer planes repeat more halo work per plane)
    long long want = (tiles * c->np + 4095) / 4096;
    int cp = (int)std::max<long long>(8, want);
    return std::min(cp, c->np);
}

template <class R> StepArgs<R> step_args(lbm_ctx *c, const Coefs<R> &cf, const void *src, void *dst,
                                         int write, int observe, double *orho, double *ovel)
{
    StepArgs<R> a{};
    a.src = src;
    a.dst = dst;
    a.obs_rho = orho;
    a.obs_vel = ovel;
    a.nx = c->nx;
    a.ny = c->ny;
    a.np = c->np;
    a.n = c->n;
    a.cp = c->cp;
    grid_of(c, c->tile, c->cp, a.tiles_x, a.tiles_y, a.chunks);
    a.write_pops = write;
    a.observe = observe;
    a.c = cf;
    return a;
}

template <class L, int SCH, class S, class R, int TX, int TY>
void launch_one(lbm_ctx *c, const StepArgs<R> &a)
{
    int nb = a.tiles_x * a.tiles_y * a.chunks;
    step_kernel<L, SCH, S, R, TX, TY><<<nb, TX * TY, 0, c->stream>>>(a);
}

template <class L, int SCH, class S, class R>
void launch_tiles(lbm_ctx *c, const StepArgs<R> &a)
{
    if constexpr (L::DIM == 2) {
        switch (c->tile) {
        case 0: launch_one<L, SCH, S, R, 64, 1>(c, a); break;
        case 1: launch_one<L, SCH, S, R, 128, 1>(c, a); break;
        default: launch_one<L, SCH, S, R, 256, 1>(c, a); break;
        }
    } else {
        switch (c->tile) {
        case 0: launch_one<L, SCH, S, R, 64, 4>(c, a); break;
        case 1: launch_one<L, SCH, S, R, 32, 8>(c, a); break;
        case 2: launch_one<L, SCH, S, R, 64, 8>(c, a); break;
        case 3: launch_one<L, SCH, S, R, 32, 16>(c, a); break;
        default: launch_one<L, SCH, S, R, 128, 4>(c, a); break;
        }
    }
}

template <class L, int SCH>
void launch_step_l(lbm_ctx *c, const void *src, void *dst, int write, int observe, double *orho,
                   double *ovel)
{
    if (c->p.storage == LBM_STORE_F64)
        launch_tiles<L, SCH, double, double>(c, step_args(c, c->cd, src, dst, write, observe, orho, ovel));
    else if (c->p.compute == LBM_COMPUTE_F64)
        launch_tiles<L, SCH, float, double>(c, step_args(c, c->cd, src, dst, write, observe, orho, ovel));
    else
        launch_tiles<L, SCH, float, float>(c, step_args(c, c->cf, src, dst, write, observe, orho, ovel));
}

void launch_step(lbm_ctx *c, const void *src, void *dst, int write, int observe, double *orho,
                 double *ovel)
{
    bool d3 = c->p.lattice == LBM_D3Q19;
    bool fo = c->p.scheme == LBM_SCHEME_FORCE;
    if (!d3 && !fo) launch_step_l<D2Q9, SCHEME_EQ>(c, src, dst, write, observe, orho, ovel);
    if (!d3 && fo) launch_step_l<D2Q9, SCHEME_FORCE>(c, src, dst, write, observe, orho, ovel);
    if (d3 && !fo) launch_step_l<D3Q19, SCHEME_EQ>(c, src, dst, write, observe, orho, ovel);
    if (d3 && fo) launch_step_l<D3Q19, SCHEME_FORCE>(c, src, dst, write, observe, orho, ovel);
}

Geom geom(const lbm_ctx *c) { return Geom{c->nx, c->ny, c->np, c->n, c->n}; }

unsigned grid1(long long n) { return unsigned((n + 255) / 256); }

template <class L, class S> void launch_init_t(lbm_ctx *c, const double *rho0, const double *u0)
{
    if (c->p.scheme == LBM_SCHEME_EQ)
        init_kernel<L, SCHEME_EQ, S><<<grid1(c->n), 256, 0, c->stream>>>(
            geom(c), c->cd, rho0, u0, static_cast<S *>(buf_cur(c)));
    else
        init_kernel<L, SCHEME_FORCE, S><<<grid1(c->n), 256, 0, c->stream>>>(
            geom(c), c->cd, rho0, u0, static_cast<S *>(buf_cur(c)));
}

void launch_init(lbm_ctx *c, const double *rho0, const double *u0)
{
    bool d3 = c->p.lattice == LBM_D3Q19, f64 = c->p.storage == LBM_STORE_F64;
    if (!d3 && f64) launch_init_t<D2Q9, double>(c, rho0, u0);
    if (!d3 && !f64) launch_init_t<D2Q9, float>(c, rho0, u0);
    if (d3 && f64) launch_init_t<D3Q19, double>(c, rho0, u0);
    if (d3 && !f64) launch_init_t<D3Q19, float>(c, rho0, u0);
}

template <class L, class S> void state_io_t(lbm_ctx *c, double *out, const double *in)
{
    if (out)
        get_state_kernel<L, S><<<grid1(c->n), 256, 0, c->stream>>>(
            geom(c), c->cd, static_cast<const S *>(buf_cur(c)), out);
    else
        set_state_kernel<L, S><<<grid1(c->n), 256, 0, c->stream>>>(
            geom(c), c->cd, in, static_cast<S *>(buf_cur(c)));
}

void state_io(lbm_ctx *c, double *out, const double *in)
{
    bool d3 = c->p.lattice == LBM_D3Q19, f64 = c->p.storage == LBM_STORE_F64;
    if (!d3 && f64) state_io_t<D2Q9, double>(c, out, in);
    if (!d3 && !f64) state_io_t<D2Q9, float>(c, out, in);
    if (d3 && f64) state_io_t<D3Q19, double>(c, out, in);
    if (d3 && !f64) state_io_t<D3Q19, float>(c, out, in);
}

int nred_blocks(long long n) { return (int)std::min<long long>(RED_BLOCKS, (n + 255) / 256); }

constexpr unsigned long long OBS_OPS =
    (unsigned long long)RED_MAX | ((unsigned long long)RED_MAX << 2) |
    ((unsigned long long)RED_SUM << 4) | ((unsigned long long)RED_MIN << 6) |
    ((unsigned long long)RED_MAX << 8) | ((unsigned long long)RED_SUM << 10);

// reduce an observation (rho, vel, optional prev) into host out[OBS_NV]
int reduce_obs(lbm_ctx *c, const double *rho, const double *vel, const double *prev, double *out)
{
    int nb = nred_blocks(c->n);
    double *part = ws_d(c, c->lay.off_part), *res = ws_d(c, c->lay.off_res);
    reduce_obs_kernel<<<nb, RED_THREADS, 0, c->stream>>>(c->n, c->p.b, rho, vel, prev, part);
    finish_kernel<<<1, RED_THREADS, 0, c->stream>>>(nb, OBS_NV, OBS_OPS, part, res);
    if (hipGetLastError() != hipSuccess) return LBM_E_DEVICE;
    if (hipMemcpyAsync(out, res, OBS_NV * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
        hipSuccess)
        return LBM_E_DEVICE;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM_E_DEVICE;
    return LBM_OK;
}

template <class L, class S> int totals_t(lbm_ctx *c, double *mass, double *mom)
{
    constexpr int Q = L::Q;
    int nb = nred_blocks(c->n);
    double *part = ws_d(c, c->lay.off_part), *res = ws_d(c, c->lay.off_res);
    reduce_pops_kernel<L, S><<<nb, RED_THREADS, 0, c->stream>>>(
        geom(c), static_cast<const S *>(buf_cur(c)), part);
    finish_kernel<<<1, RED_THREADS, 0, c->stream>>>(nb, Q, 0ull, part, res);
    if (hipGetLastError() != hipSuccess) return LBM_E_DEVICE;
    double h[19];
    if (hipMemcpyAsync(h, res, Q * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return LBM_E_DEVICE;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM_E_DEVICE;
    double m = 0, mx = 0, my = 0, mz = 0;
    for (int i = 0; i < Q; i++) {
        m += h[i];
        mx += L::ex[i] * h[i];
        my += L::ey[i] * h[i];
        mz += L::ez[i] * h[i];
    }
    // the stored values are f_i - s_i; add back n * sum_i s_i (the shift is
    // symmetric, so it carries no momentum)
    m += double(c->n) * c->cd.shift_sum;
    if (mass) *mass = m;
    if (mom) {
        mom[0] = mx;
        mom[1] = my;
        mom[2] = mz;
    }
    return LBM_OK;
}

// van der Waals pressure p0(rho) of Eq. (p0), its derivative and the chemical
// potential, for the Maxwell construction in lbm_coexistence (bisections)
double vdw_p(double a, double b, double T, double r) { return r * T / (1 - b * r) - a * r * r; }
double vdw_dp(double a, double b, double T, double r)
{
    return T / ((1 - b * r) * (1 - b * r)) - 2 * a * r;
}
double vdw_mu(double a, double b, double T, double r)
{
    return T * std::log(r / (1 - b * r)) + T / (1 - b * r) - 2 * a * r;
}

// Streaming copy, 16 bytes per thread, one pass (one thread per 16 bytes,
// non-temporal stores): the achievable HBM rate for one read and one write
// of every byte, against which the step kernels' algorithmic traffic is
// compared.  Measured on 1.275 GB: one pass 6.36 TB/s; the same with plain
// stores 6.19; four 16-byte loads per thread 5.71; a grid-stride loop over
// 16k workgroups 5.09; hipMemcpy device to device 5.17.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void stream_copy_kernel(const f32x4 *__restrict__ src,
                                                          f32x4 *__restrict__ dst, long long n16)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n16) __builtin_nontemporal_store(src[k], &dst[k]);
}

} // namespace

extern "C" {

int lbm_stream_copy(const void *dev_src, void *dev_dst, size_t bytes, void *stream)
{
    if (!dev_src || !dev_dst || bytes % 16 || (reinterpret_cast<uintptr_t>(dev_src) |
                                               reinterpret_cast<uintptr_t>(dev_dst)) % 16)
        return LBM_E_INVAL;
    const long long n16 = (long long)(bytes / 16);
    if (n16 == 0) return LBM_OK;
    if ((n16 + 255) / 256 >= (1ll << 31)) return LBM_E_INVAL;
    const unsigned blocks = unsigned((n16 + 255) / 256);
    stream_copy_kernel<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const f32x4 *>(dev_src), static_cast<f32x4 *>(dev_dst), n16);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

void lbm_params_default(lbm_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->a = 9.0 / 49.0;
    p->b = 2.0 / 21.0;
    p->T = 0.56;
    p->kappa = 0.025;
    p->tau = 1.0;
    p->lattice = LBM_D2Q9;
    p->scheme = LBM_SCHEME_EQ;
    p->storage = LBM_STORE_F64;
    p->nx = 100;
    p->ny = 100;
    p->nz = 1;
    p->B = p->D = p->F = NAN;
    p->wp_diag = p->wt_diag = p->wxx_diag = NAN;
    p->galilean_lambda = 1;
    p->shift_mode = LBM_SHIFT_REST_EQ;
    p->rho_shift = NAN;
    p->tile = -1;
    p->planes_per_block = 0;
    p->compute = LBM_COMPUTE_NATIVE;
}

size_t lbm_workspace_bytes(const lbm_params *p)
{
    if (!valid_params(p)) return 0;
    return layout(p).total;
}

const char *lbm_strerror(int code)
{
    switch (code) {
    case LBM_OK: return "ok";
    case LBM_E_INVAL: return "invalid argument or unphysical parameter";
    case LBM_E_NOMEM: return "workspace smaller than lbm_workspace_bytes()";
    case LBM_E_DEVICE: return "HIP call or kernel launch failed";
    case LBM_E_NONFINITE: return "non-finite state or b*rho >= 1";
    case LBM_E_STATE: return "call not valid in the current state";
    case LBM_E_LIMIT: return "input beyond the fixed scratch of an allocation-free call";
    default: return "unknown status";
    }
}

int lbm_init(lbm_ctx **out, const lbm_params *p, void *dev_workspace, size_t bytes, void *stream,
             const double *dev_rho0, const double *dev_u0)
{
    if (!out || !valid_params(p) || !dev_workspace || !dev_rho0) return LBM_E_INVAL;
    *out = nullptr;
    Layout lay = layout(p);
    if (bytes < lay.total) return LBM_E_NOMEM;
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN) return LBM_E_INVAL;
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_E_NOMEM;
    c->p = *p;
    c->lay = lay;
    c->ws = static_cast<char *>(dev_workspace);
    c->stream = static_cast<hipStream_t>(stream);
    c->cur = 0;
    c->steps = 0;
    c->prev_valid = false;
    if (p->lattice == LBM_D2Q9) {
        c->nx = p->nx; c->ny = 1; c->np = p->ny;
    } else {
        c->nx = p->nx; c->ny = p->ny; c->np = p->nz;
    }
    c->n = (long long)p->nx * p->ny * p->nz;
    c->tile = p->tile >= 0 ? p->tile : default_tile(p);
    c->cp = p->planes_per_block > 0 ? std::min(p->planes_per_block, c->np) : default_planes(c, c->tile);
    c->cd = make_coefs(p);
    // validate the initial density: finite, 0 < rho < 1/b; get its mean
    double obs[OBS_NV];
    int rc = reduce_obs(c, dev_rho0, nullptr, nullptr, obs);
    if (rc != LBM_OK) {
        delete c;
        return rc;
    }
    if (obs[2] != 0.0) {
        delete c;
        return LBM_E_INVAL;
    }
    double mean = obs[5] / double(c->n);
    double rs = std::isnan(p->rho_shift) ? mean : p->rho_shift;
    if (p->storage != LBM_STORE_F64 && !(rs > 0.0 && p->b * rs < 1.0)) {
        delete c;
        return LBM_E_INVAL;
    }
    make_shift(p, c->cd, rs);
    c->cf = to_float(c->cd, p->lattice);
    launch_init(c, dev_rho0, dev_u0);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        delete c;
        return LBM_E_DEVICE;
    }
    *out = c;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, long long nsteps)
{
    if (!c || nsteps < 0) return LBM_E_INVAL;
    for (long long s = 0; s < nsteps; s++) {
        launch_step(c, buf_cur(c), buf_nxt(c), 1, 0, nullptr, nullptr);
        c->cur ^= 1;
        c->steps++;
    }
    if (nsteps) c->prev_valid = false;
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_moments(lbm_ctx *c, double *dev_rho, double *dev_vel)
{
    if (!c) return LBM_E_INVAL;
    double *r = dev_rho ? dev_rho : ws_d(c, c->lay.off_rho);
    double *v = dev_vel ? dev_vel : ws_d(c, c->lay.off_vel);
    launch_step(c, buf_cur(c), nullptr, 0, 1, r, v);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_max_spurious_u(lbm_ctx *c, double *host_out)
{
    if (!c || !host_out) return LBM_E_INVAL;
    double *r = ws_d(c, c->lay.off_rho), *v = ws_d(c, c->lay.off_vel);
    launch_step(c, buf_cur(c), nullptr, 0, 1, r, v);
    if (hipGetLastError() != hipSuccess) return LBM_E_DEVICE;
    double obs[OBS_NV];
    int rc = reduce_obs(c, r, v, nullptr, obs);
    if (rc != LBM_OK) return rc;
    *host_out = obs[0];
    return obs[2] != 0.0 ? LBM_E_NONFINITE : LBM_OK;
}

int lbm_invariants(lbm_ctx *c, double *host_mass, double *host_mom)
{
    if (!c) return LBM_E_INVAL;
    bool d3 = c->p.lattice == LBM_D3Q19, f64 = c->p.storage == LBM_STORE_F64;
    if (!d3 && f64) return totals_t<D2Q9, double>(c, host_mass, host_mom);
    if (!d3 && !f64) return totals_t<D2Q9, float>(c, host_mass, host_mom);
    if (d3 && f64) return totals_t<D3Q19, double>(c, host_mass, host_mom);
    return totals_t<D3Q19, float>(c, host_mass, host_mom);
}

int lbm_step_observed(lbm_ctx *c, long long nsteps, double *host_residual, double *host_max_vel)
{
    if (!c || nsteps < 1) return LBM_E_INVAL;
    int rc = lbm_step(c, nsteps - 1);
    if (rc != LBM_OK) return rc;
    double *r = ws_d(c, c->lay.off_rho), *v = ws_d(c, c->lay.off_vel);
    double *pv = ws_d(c, c->lay.off_prev);
    // last step: observe the state it starts from into `prev` ...
    launch_step(c, buf_cur(c), buf_nxt(c), 1, 1, r, pv);
    c->cur ^= 1;
    c->steps++;
    // ... and the state it produces into `vel`
    launch_step(c, buf_cur(c), nullptr, 0, 1, r, v);
    if (hipGetLastError() != hipSuccess) return LBM_E_DEVICE;
    double obs[OBS_NV];
    rc = reduce_obs(c, r, v, pv, obs);
    if (rc != LBM_OK) return rc;
    if (host_residual) *host_residual = obs[1];
    if (host_max_vel) *host_max_vel = obs[0];
    return obs[2] != 0.0 ? LBM_E_NONFINITE : LBM_OK;
}

int lbm_get_state(lbm_ctx *c, double *dev_f)
{
    if (!c || !dev_f) return LBM_E_INVAL;
    state_io(c, dev_f, nullptr);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_set_state(lbm_ctx *c, const double *dev_f)
{
    if (!c || !dev_f) return LBM_E_INVAL;
    state_io(c, nullptr, dev_f);
    c->prev_valid = false;
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

long long lbm_steps_done(const lbm_ctx *c) { return c ? c->steps : -1; }

int lbm_shift(const lbm_ctx *c, double *host_shift)
{
    if (!c || !host_shift) return LBM_E_INVAL;
    for (int i = 0; i < c->p.lattice; i++)
        host_shift[i] = c->cd.shift[i];
    return LBM_OK;
}

int lbm_tile_count(int lattice)
{
    if (lattice == LBM_D2Q9) return NT2;
    if (lattice == LBM_D3Q19) return NT3;
    return LBM_E_INVAL;
}

int lbm_tile_shape(int lattice, int k, int *tile_x, int *tile_y)
{
    int nt = lbm_tile_count(lattice);
    if (nt < 0 || k < 0 || k >= nt || !tile_x || !tile_y) return LBM_E_INVAL;
    TileShape t = tile_shape(lattice, k);
    *tile_x = t.tx;
    *tile_y = t.ty;
    return LBM_OK;
}

int lbm_set_launch(lbm_ctx *c, int tile, int planes)
{
    if (!c) return LBM_E_INVAL;
    if (tile >= lbm_tile_count(c->p.lattice)) return LBM_E_INVAL;
    if (tile >= 0) c->tile = tile;
    if (planes > 0) c->cp = std::min(planes, c->np);
    return LBM_OK;
}

int lbm_get_launch(const lbm_ctx *c, int *tile, int *planes, int *workgroups)
{
    if (!c) return LBM_E_INVAL;
    if (tile) *tile = c->tile;
    if (planes) *planes = c->cp;
    if (workgroups) {
        int a, b, ch;
        grid_of(c, c->tile, c->cp, a, b, ch);
        *workgroups = a * b * ch;
    }
    return LBM_OK;
}

int lbm_destroy(lbm_ctx *c)
{
    delete c;
    return LBM_OK;
}

int lbm_coexistence(double a, double b, double T, double *rho_gas, double *rho_liq)
{
    if (!rho_gas || !rho_liq || !(a > 0) || !(b > 0) || !(T > 0)) return LBM_E_INVAL;
    const double Tc = 8.0 * a / (27.0 * b), rc = 1.0 / (3.0 * b), rmax = 1.0 / b;
    if (!(T < Tc)) return LBM_E_INVAL;
    // Spinodals sg < rc < sl (dp/drho = 0), by bisection on the sign of dp/drho.
    // (Each bisection stops once the midpoint is no longer strictly inside
    // the interval: the two ends are adjacent doubles.)
    auto spin = [&](double lo, double hi) {
        const bool up = vdw_dp(a, b, T, lo) > 0;
        for (int k = 0; k < 2100; k++) {
            const double m = 0.5 * (lo + hi);
            if (!(lo < m && m < hi)) break;
            if ((vdw_dp(a, b, T, m) > 0) == up) lo = m; else hi = m;
        }
        return 0.5 * (lo + hi);
    };
    const double sg = spin(0.0, rc), sl = spin(rc, rmax);
    if (!(0.0 < sg && sg < rc && rc < sl && sl < rmax)) return LBM_E_INVAL;
    // mu increases with rho on both stable branches (d mu / d rho = (dp/drho)
    // / rho > 0), so the density with a given mu is found by bisection on
    // each: the gas branch (0, sg) and the liquid branch (sl, 1/b).
    auto on_branch = [&](double mu, double lo, double hi) {
        for (int k = 0; k < 2100; k++) {
            const double m = 0.5 * (lo + hi);
            if (!(lo < m && m < hi)) break;
            if (vdw_mu(a, b, T, m) < mu) lo = m; else hi = m;
        }
        return 0.5 * (lo + hi);
    };
    // Maxwell construction: the common mu of the two phases makes their
    // pressures equal.  Between mu(sl) and mu(sg), p(liquid) - p(gas) rises
    // from negative to positive; bisect on mu.
    double mlo = vdw_mu(a, b, T, sl), mhi = vdw_mu(a, b, T, sg);
    if (!(mlo < mhi)) return LBM_E_INVAL;
    double g = 0.0, l = 0.0;
    for (int k = 0; k < 2100; k++) {
        const double m = 0.5 * (mlo + mhi);
        g = on_branch(m, 0.0, sg);
        l = on_branch(m, sl, rmax);
        if (!(mlo < m && m < mhi)) break;
        if (vdw_p(a, b, T, l) - vdw_p(a, b, T, g) < 0) mlo = m; else mhi = m;
    }
    // the result must be a coexistence point, not just the end of the search
    const double pg = vdw_p(a, b, T, g), pl = vdw_p(a, b, T, l);
    const double ug = vdw_mu(a, b, T, g), ul = vdw_mu(a, b, T, l);
    const double pscale = std::fabs(vdw_p(a, b, T, sg)) + std::fabs(vdw_p(a, b, T, sl)) + T * rc;
    if (!(0.0 < g && g < sg && sl < l && l < rmax) || !(std::fabs(pl - pg) <= 1e-9 * pscale) ||
        !(std::fabs(ul - ug) <= 1e-9 * (std::fabs(ug) + T)))
        return LBM_E_INVAL;
    *rho_gas = g;
    *rho_liq = l;
    return LBM_OK;
}

} // extern "C"

#include "lbm_batch_host.h"
#include "lbm_net_host.h"
#include "lbm_binary_host.h"
