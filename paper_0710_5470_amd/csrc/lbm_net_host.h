// lbm_net_host.h -- host side of the warm-start network kernels (included
// once, at the end of lbm_capi.hip).

#include <mutex>

#include "lbm_net.h"
#include "lbm_warm.h"

// Device scratch of lbm_net_conv3x3_bwd_weight_noalloc: the per-workgroup
// partials of the weight gradient.  Every GPU holds its own copy at its own
// address; host code never passes this name to a kernel (on the host it is
// only a stand-in for the symbol) but the address that hipGetSymbolAddress
// returns for the current device.
constexpr size_t NET_SCRATCH_BYTES = size_t(16) << 20;
static __device__ __align__(256) float scratch[NET_SCRATCH_BYTES / sizeof(float)];

namespace {

constexpr int NET_SCRATCH_DEVICES = 64;
std::mutex net_scratch_mu;
void *net_scratch_ptr[NET_SCRATCH_DEVICES];  // per device, looked up once

// Device address of `scratch` on the current device (looked up on the
// first call on that device, with that device current).
int net_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NET_SCRATCH_DEVICES) return LBM_E_DEVICE;
    std::lock_guard<std::mutex> lock(net_scratch_mu);
    if (!net_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LBM_E_DEVICE;
        net_scratch_ptr[dev] = p;
    }
    *out = net_scratch_ptr[dev];
    return LBM_OK;
}

bool conv_ok(const lbm_conv_shape *s)
{
    if (!s || s->nb < 1 || s->h < 1 || s->w < 1) return false;
    if (s->cin < 16 || s->cin > 32 || s->cin % 16) return false;
    if (s->cout < 16 || s->cout > 32 || s->cout % 16) return false;
    if (s->cout_real < 1 || s->cout_real > s->cout) return false;
    long long npix = (long long)s->nb * s->h * s->w;
    return npix % 16 == 0 && npix <= 0x7FFFFFFFLL;  // 32-bit pixel indices in the kernels
}

lbmnet::ConvShape conv_shape(const lbm_conv_shape *s)
{
    return lbmnet::ConvShape{s->nb, s->h, s->w, s->cin, s->cout, s->cout_real};
}

bool aligned16(const void *p) { return p && (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

constexpr int NET_CHUNK = 1024;  // pixels per workgroup in the weight gradient

unsigned conv_grid(const lbm_conv_shape *s)
{
    long long npix = (long long)s->nb * s->h * s->w;
    const long long per_wg = 4LL * 16 * lbmnet::CONV_MT;  // 4 waves of CONV_MT 16-pixel tiles
    return unsigned((npix + per_wg - 1) / per_wg);
}

} // namespace

extern "C" {

int lbm_net_conv3x3_fwd(const lbm_conv_shape *s, const float *dev_in, int relu_in, const float *dev_w,
                        const float *dev_b, float *dev_out, void *stream)
{
    if (!conv_ok(s) || !aligned16(dev_in) || !aligned16(dev_w) || !dev_b || !dev_out) return LBM_E_INVAL;
    lbmnet::conv_fwd_kernel<<<conv_grid(s), lbmnet::NET_THREADS, 0, static_cast<hipStream_t>(stream)>>>(
        conv_shape(s), dev_in, relu_in, dev_w, dev_b, dev_out);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_net_conv3x3_bwd_data(const lbm_conv_shape *s, const float *dev_dout, const float *dev_w,
                             const float *dev_zin, float *dev_din, void *stream)
{
    if (!conv_ok(s) || !aligned16(dev_dout) || !dev_w || !dev_din) return LBM_E_INVAL;
    lbmnet::conv_bwd_data_kernel<<<conv_grid(s), lbmnet::NET_THREADS, 0, static_cast<hipStream_t>(stream)>>>(
        conv_shape(s), dev_dout, dev_w, dev_zin, dev_din);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

size_t lbm_net_conv3x3_bwd_weight_workspace(const lbm_conv_shape *s)
{
    if (!conv_ok(s)) return 0;
    long long npix = (long long)s->nb * s->h * s->w;
    long long parts = (npix + NET_CHUNK - 1) / NET_CHUNK;
    return size_t(parts) * (9 * s->cout * s->cin + s->cout) * sizeof(float);
}

} // extern "C"

namespace {

// Weight gradient with the per-workgroup partials in `part` (at least
// lbm_net_conv3x3_bwd_weight_workspace(s) bytes): one workgroup per
// NET_CHUNK pixels, then a fixed-order sum of the partials.
int bwd_weight_launch(const lbm_conv_shape *s, const float *dev_dout, const float *dev_in, int relu_in,
                      float *dev_dw, float *dev_db, float *part, hipStream_t st)
{
    long long npix = (long long)s->nb * s->h * s->w;
    int parts = int((npix + NET_CHUNK - 1) / NET_CHUNK);
    lbmnet::conv_bwd_weight_kernel<<<parts, lbmnet::NET_THREADS, 0, st>>>(conv_shape(s), dev_dout, dev_in,
                                                                          relu_in, NET_CHUNK, part);
    const int nw = 9 * s->cout * s->cin;
    const int len = nw + s->cout;  // weight gradient, then bias gradient
    lbmnet::sum_parts_kernel<<<(len + 63) / 64, 256, 0, st>>>(parts, len, nw, part, dev_dw, dev_db);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

} // namespace

extern "C" {

int lbm_net_conv3x3_bwd_weight(const lbm_conv_shape *s, const float *dev_dout, const float *dev_in,
                               int relu_in, float *dev_dw, float *dev_db, void *dev_ws, size_t ws_bytes,
                               void *stream)
{
    if (!conv_ok(s) || !dev_dout || !dev_in || !dev_dw || !dev_db || !dev_ws) return LBM_E_INVAL;
    if (ws_bytes < lbm_net_conv3x3_bwd_weight_workspace(s)) return LBM_E_NOMEM;
    return bwd_weight_launch(s, dev_dout, dev_in, relu_in, dev_dw, dev_db, static_cast<float *>(dev_ws),
                             static_cast<hipStream_t>(stream));
}

int lbm_net_conv3x3_bwd_weight_noalloc(const lbm_conv_shape *s, const float *dev_dout, const float *dev_in,
                                       int relu_in, float *dev_dw, float *dev_db, void *stream)
{
    if (!conv_ok(s) || !dev_dout || !dev_in || !dev_dw || !dev_db) return LBM_E_INVAL;
    if (lbm_net_conv3x3_bwd_weight_workspace(s) > NET_SCRATCH_BYTES) return LBM_E_LIMIT;
    void *part = nullptr;
    int rc = net_scratch(&part);
    if (rc != LBM_OK) return rc;
    return bwd_weight_launch(s, dev_dout, dev_in, relu_in, dev_dw, dev_db, static_cast<float *>(part),
                             static_cast<hipStream_t>(stream));
}

int lbm_net_mse(long long npix, int c, int creal, const float *dev_pred, const float *dev_target,
                float *dev_grad, double *dev_part, double *host_loss, void *stream)
{
    if (npix < 1 || c < 1 || creal < 1 || creal > c || !dev_pred || !dev_target || !dev_grad || !dev_part)
        return LBM_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nblk = 1024;
    lbmnet::mse_kernel<<<nblk, lbmnet::NET_THREADS, 0, st>>>(npix, c, creal, dev_pred, dev_target, dev_grad,
                                                             dev_part);
    if (hipGetLastError() != hipSuccess) return LBM_E_DEVICE;
    if (host_loss) {
        double h[nblk];
        if (hipMemcpyAsync(h, dev_part, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return LBM_E_DEVICE;
        double a = 0.0;
        for (int k = 0; k < nblk; k++) a += h[k];
        *host_loss = a;
    }
    return LBM_OK;
}

int lbm_net_adam(int n, float *dev_p, const float *dev_g, float *dev_m, float *dev_v, double lr, double b1,
                 double b2, double eps, long long t, void *stream)
{
    if (n < 1 || !dev_p || !dev_g || !dev_m || !dev_v || t < 1) return LBM_E_INVAL;
    double c1 = 1.0 - std::pow(b1, double(t)), c2 = 1.0 - std::pow(b2, double(t));
    lbmnet::adam_kernel<<<(n + 255) / 256, 256, 0, static_cast<hipStream_t>(stream)>>>(
        n, dev_p, dev_g, dev_m, dev_v, float(lr), float(b1), float(b2), float(eps), float(c1), float(c2));
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_warm_features(int nprob, int side, const double *dev_consts, const double *dev_rho0, double rho_mean,
                      double rho_scale, float *dev_x, void *stream)
{
    if (nprob < 1 || side < 1 || !dev_consts || !dev_rho0 || !aligned16(dev_x) || !(rho_scale != 0.0))
        return LBM_E_INVAL;
    const long long total = (long long)nprob * side * side;
    const unsigned grid = unsigned(std::min<long long>((total + 255) / 256, 65536));
    lbmwarm::warm_features_kernel<<<grid, 256, 0, static_cast<hipStream_t>(stream)>>>(
        nprob, side, dev_consts, dev_rho0, rho_mean, rho_scale, dev_x);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_warm_targets(long long ntot, const double *dev_rho, const double *dev_rho0, const double *dev_vel,
                     double s_rho, double s_u, float *dev_y, void *stream)
{
    if (ntot < 1 || !dev_rho || !dev_rho0 || !dev_vel || !aligned16(dev_y) || !(s_rho != 0.0) || !(s_u != 0.0))
        return LBM_E_INVAL;
    const unsigned grid = unsigned(std::min<long long>((ntot + 255) / 256, 65536));
    lbmwarm::warm_targets_kernel<<<grid, 256, 0, static_cast<hipStream_t>(stream)>>>(ntot, dev_rho, dev_rho0,
                                                                                    dev_vel, s_rho, s_u, dev_y);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_warm_project(int nprob, int side, int cpad, const float *dev_pred, const double *dev_rho0, double s_rho,
                     double s_u, int with_velocity, int symmetrize, double rho_lo, double rho_hi, double *dev_rho,
                     double *dev_u, void *stream)
{
    if (nprob < 1 || side < 1 || cpad < (with_velocity ? 3 : 1) || !dev_pred || !dev_rho0 || !dev_rho ||
        !dev_u || !(rho_lo < rho_hi))
        return LBM_E_INVAL;
    const long long ntot = (long long)nprob * side * side;
    lbmwarm::warm_project_kernel<<<nprob, lbmwarm::WARM_THREADS, 0, static_cast<hipStream_t>(stream)>>>(
        side, cpad, dev_pred, dev_rho0, s_rho, s_u, with_velocity, symmetrize, rho_lo, rho_hi, dev_rho, dev_u,
        ntot);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

} // extern "C"
