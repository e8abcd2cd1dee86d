// lbm_binary_host.h -- host side of the binary-fluid stepper (included once,
// at the end of lbm_capi.hip, so it shares that file's reduction helpers).
//
// A context owns no device memory: the caller's workspace holds the f and g
// population buffers (two each, ping-pong), the observation fields and the
// reduction partials.

#include "lbm_binary.h"

struct lbm_bin_ctx {
    lbm_bin_params p;
    hipStream_t stream;
    char *ws;
    size_t o_fa, o_fb, o_ga, o_gb, o_rho, o_phi, o_vel, o_T, o_force, o_part, o_res, total;
    int cur;            // 0: state in (fa, ga), 1: in (fb, gb)
    long long steps;
    int tile, cp;
    int nx, ny, np;     // kernel geometry
    long long n;
    BinCoefs c;
};

namespace {

// launch shapes: D2Q9 rows of tx sites; D3Q19 tx x ty in-plane tiles
constexpr TileShape BIN_TILES_2D[] = {{128, 1}, {256, 1}};
constexpr TileShape BIN_TILES_3D[] = {{32, 8}, {64, 4}, {64, 8}, {128, 4}};
constexpr int BNT2 = sizeof(BIN_TILES_2D) / sizeof(BIN_TILES_2D[0]);
constexpr int BNT3 = sizeof(BIN_TILES_3D) / sizeof(BIN_TILES_3D[0]);

TileShape bin_tile(int lattice, int k) { return lattice == LBM_D2Q9 ? BIN_TILES_2D[k] : BIN_TILES_3D[k]; }
int bin_tile_count(int lattice) { return lattice == LBM_D2Q9 ? BNT2 : BNT3; }

// call f with a value of the velocity-set type of `lattice`
template <class F> void bin_dispatch(int lattice, F &&f)
{
    if (lattice == LBM_D2Q9) f(D2Q9{});
    else if (lattice == LBM_D3Q19) f(D3Q19{});
    else f(D3Q15{});
}

bool bin_valid(const lbm_bin_params *p)
{
    if (!p) return false;
    if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q19 && p->lattice != LBM_D3Q15) return false;
    if (p->lattice == LBM_D3Q15 && p->scheme != LBM_SCHEME_EQ) return false;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
    if (p->lattice == LBM_D2Q9 && p->nz != 1) return false;
    if ((double)p->nx * p->ny * p->nz * p->lattice >= 4294967296.0) return false;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return false;
    if (!(p->tau_phi > 0.5) || !std::isfinite(p->tau_phi)) return false;
    if (!std::isfinite(p->phi_a) || !(p->phi_b >= 0.0) || !std::isfinite(p->phi_b)) return false;
    if (!(p->kappa >= 0.0) || !std::isfinite(p->kappa)) return false;
    if (!(p->gamma >= 0.0) || !std::isfinite(p->gamma)) return false;
    if (p->tile >= bin_tile_count(p->lattice)) return false;
    if (p->wall != 0 && p->wall != 1) return false;
    if (p->scheme != LBM_SCHEME_EQ && p->scheme != LBM_SCHEME_FORCE) return false;
    if (p->lattice == LBM_D3Q19 &&
        (!std::isnan(p->wp_diag) || !std::isnan(p->wt_diag) || !std::isnan(p->wxx_diag)))
        return false;
    for (double v : {p->B, p->D, p->wp_diag, p->wt_diag, p->wxx_diag})
        if (std::isinf(v)) return false;
    return true;
}

void bin_layout(lbm_bin_ctx *c)
{
    const size_t n = (size_t)c->p.nx * c->p.ny * c->p.nz;
    const size_t pops = align_up(n * c->p.lattice * 8);
    size_t o = 0;
    c->o_fa = o; o += pops;
    c->o_fb = o; o += pops;
    c->o_ga = o; o += pops;
    c->o_gb = o; o += pops;
    c->o_rho = o; o += align_up(n * 8);
    c->o_phi = o; o += align_up(n * 8);
    c->o_vel = o; o += align_up(3 * n * 8);
    const size_t nf = c->p.scheme == LBM_SCHEME_FORCE ? n : 0;  // forcing scheme only
    c->o_T = o; o += align_up(3 * nf * 8);  // d phi
    c->o_force = o; o += align_up(3 * nf * 8);
    c->o_part = o; o += align_up((size_t)RED_BLOCKS * 20 * 8);
    c->o_res = o; o += align_up(32 * 8);
    c->total = o;
}

double *bws(lbm_bin_ctx *c, size_t off) { return reinterpret_cast<double *>(c->ws + off); }
double *bin_f(lbm_bin_ctx *c, int which) { return bws(c, which ? c->o_fb : c->o_fa); }
double *bin_g(lbm_bin_ctx *c, int which) { return bws(c, which ? c->o_gb : c->o_ga); }

// Stencils of Eqs. (xderiv), (laplace), (laplacian3d) and the equilibrium
// weights (summary / Eq. (3dres)): the paper's optimum unless overridden.
BinCoefs bin_coefs(const lbm_bin_params *p)
{
    if (p->lattice == LBM_D3Q15) {
        // D3Q15 (see the header): corner coefficients, faces from the moments
        BinCoefs c{};
        c.B = pick(p->B, 1.0 / 24.0);
        c.D = pick(p->D, 1.0 / 12.0);
        c.A = (1.0 - 8.0 * c.B) / 2.0;  // 2A + 8B = 1
        c.C = 1.0 - 4.0 * c.D;          // C + 4D = 1
        c.w_ax = 1.0 / 3.0;
        c.w_off = 1.0 / 24.0;
        c.wp_off = pick(p->wp_diag, 1.0 / 24.0);
        c.wp_ax = 0.5 - 4.0 * c.wp_off;
        c.wt_off = pick(p->wt_diag, 1.0 / 24.0);
        c.wt_ax = 0.5 - 4.0 * c.wt_off;
        const double wc = pick(p->wxx_diag, 0.0);
        c.wm_para = 0.25 - 4.0 * wc;
        c.wm_perp = -0.25 - 4.0 * wc;
        c.wm_in = wc;
        c.wm_out = 0.0;
        c.kappa = p->kappa;
        c.omega = 1.0 / p->tau;
        c.omega_g = 1.0 / p->tau_phi;
        c.pa = p->phi_a;
        c.pb = p->phi_b;
        c.gamma = p->gamma;
        return c;
    }
    lbm_params q;
    lbm_params_default(&q);
    q.lattice = p->lattice;
    q.kappa = p->kappa;
    q.tau = p->tau;
    q.B = p->B;
    q.D = p->D;
    q.wp_diag = p->wp_diag;
    q.wt_diag = p->wt_diag;
    q.wxx_diag = p->wxx_diag;
    const Coefs<double> k = make_coefs(&q);
    BinCoefs c{};
    c.A = k.A; c.B = k.B; c.C = k.C; c.D = k.D;
    c.w_ax = k.w_ax; c.w_off = k.w_off;
    c.wp_ax = k.wp_ax; c.wp_off = k.wp_off;
    c.wt_ax = k.wt_ax; c.wt_off = k.wt_off;
    c.wm_para = k.wm_para; c.wm_perp = k.wm_perp; c.wm_in = k.wm_in; c.wm_out = k.wm_out;
    c.kappa = p->kappa;
    c.omega = 1.0 / p->tau;
    c.omega_g = 1.0 / p->tau_phi;
    c.pa = p->phi_a;
    c.pb = p->phi_b;
    c.gamma = p->gamma;
    c.Ef = k.Ef;
    c.Ff = k.Ff;
    return c;
}

Geom bin_geom(const lbm_bin_ctx *c) { return Geom{c->nx, c->ny, c->np, c->n, c->n}; }

void bin_grid(const lbm_bin_ctx *c, int tile, int cp, int &tx_n, int &ty_n, int &chunks)
{
    TileShape t = bin_tile(c->p.lattice, tile);
    tx_n = (c->nx + t.tx - 1) / t.tx;
    ty_n = (c->ny + t.ty - 1) / t.ty;
    chunks = (c->np + cp - 1) / cp;
}

// planes per workgroup: enough chunks for about 1024 (D2Q9) or 512 (D3Q19)
// workgroups, but at least 8 planes each (every chunk forms phi on two
// extra planes first)
int bin_default_planes(const lbm_bin_ctx *c, int tile)
{
    int a, b, ch;
    bin_grid(c, tile, c->np, a, b, ch);
    const long long tiles = (long long)a * b, target = c->p.lattice == LBM_D2Q9 ? 1024 : 512;
    long long want = std::max<long long>(1, std::min<long long>(c->np, (target + tiles - 1) / tiles));
    return std::min(c->np, std::max(8, (int)((c->np + want - 1) / want)));
}

template <class L, int TX, int TY> void bin_launch_t(lbm_bin_ctx *c, const BinArgs &a, int nblk)
{
    if constexpr (L::Q != 15)  // no forcing scheme on D3Q15
        if (c->p.scheme == LBM_SCHEME_FORCE) {
            if (c->p.wall)
                bin_force_step_kernel<L, TX, TY, true><<<nblk, TX * TY, 0, c->stream>>>(a);
            else
                bin_force_step_kernel<L, TX, TY, false><<<nblk, TX * TY, 0, c->stream>>>(a);
            return;
        }
    if (c->p.wall)
        bin_step_kernel<L, TX, TY, true><<<nblk, TX * TY, 0, c->stream>>>(a);
    else
        bin_step_kernel<L, TX, TY, false><<<nblk, TX * TY, 0, c->stream>>>(a);
}

// Forcing scheme, for observables: the body force of the current state into
// the workspace (phi field, its gradient, the divergence of the stress);
// returns the force field, or nullptr for the equilibrium scheme.
const double *bin_body_force(lbm_bin_ctx *c)
{
    if (c->p.scheme != LBM_SCHEME_FORCE) return nullptr;
    double *phi = bws(c, c->o_phi), *T = bws(c, c->o_T), *force = bws(c, c->o_force);
    const Geom g = bin_geom(c);
    bin_dispatch(c->p.lattice, [&](auto l) {
        using L = decltype(l);
        if constexpr (L::Q != 15) {
            const bool w = c->p.wall != 0;
            if (w) bin_phi_kernel<L, true><<<grid1(c->n), 256, 0, c->stream>>>(g, bin_g(c, c->cur), phi);
            else bin_phi_kernel<L, false><<<grid1(c->n), 256, 0, c->stream>>>(g, bin_g(c, c->cur), phi);
            bin_gradient_kernel<L><<<grid1(c->n), 256, 0, c->stream>>>(g, c->c, w, phi, T);
            bin_divergence_kernel<L><<<grid1(c->n), 256, 0, c->stream>>>(g, c->c, w, T, force);
        }
    });
    return force;
}

void bin_launch_step(lbm_bin_ctx *c)
{
    BinArgs a{};
    a.c = c->c;
    a.fsrc = bin_f(c, c->cur);
    a.gsrc = bin_g(c, c->cur);
    a.fdst = bin_f(c, c->cur ^ 1);
    a.gdst = bin_g(c, c->cur ^ 1);
    a.nx = c->nx;
    a.ny = c->ny;
    a.np = c->np;
    a.stride = c->n;
    int chunks;
    bin_grid(c, c->tile, c->cp, a.tiles_x, a.tiles_y, chunks);
    a.cp = c->cp;
    if (c->p.scheme == LBM_SCHEME_FORCE) {
        // the phi field of the state; the march forms gradient and force itself
        double *phi = bws(c, c->o_phi);
        bin_dispatch(c->p.lattice, [&](auto l) {
            using L = decltype(l);
            if constexpr (L::Q != 15) {
                if (c->p.wall)
                    bin_phi_kernel<L, true><<<grid1(c->n), 256, 0, c->stream>>>(bin_geom(c), bin_g(c, c->cur), phi);
                else
                    bin_phi_kernel<L, false><<<grid1(c->n), 256, 0, c->stream>>>(bin_geom(c), bin_g(c, c->cur), phi);
            }
        });
        a.phi = phi;
    }
    const int nblk = a.tiles_x * a.tiles_y * chunks;
    bin_dispatch(c->p.lattice, [&](auto l) {
        using L = decltype(l);
        if constexpr (L::DIM == 2) {
            if (c->tile == 0) bin_launch_t<L, 128, 1>(c, a, nblk);
            else bin_launch_t<L, 256, 1>(c, a, nblk);
        } else {
            if (c->tile == 0) bin_launch_t<L, 32, 8>(c, a, nblk);
            else if (c->tile == 1) bin_launch_t<L, 64, 4>(c, a, nblk);
            else if (c->tile == 2) bin_launch_t<L, 64, 8>(c, a, nblk);
            else bin_launch_t<L, 128, 4>(c, a, nblk);
        }
    });
}

void bin_launch_moments(lbm_bin_ctx *c, double *rho, double *phi, double *vel)
{
    const double *force = vel ? bin_body_force(c) : nullptr;
    bin_dispatch(c->p.lattice, [&](auto l) {
        bin_moments_kernel<decltype(l)><<<grid1(c->n), 256, 0, c->stream>>>(
            bin_geom(c), c->p.wall, bin_f(c, c->cur), bin_g(c, c->cur), force, rho, phi, vel);
    });
}

// reduce (rho, vel) into out[OBS_NV] (b = 0: a site is bad if non-finite or rho <= 0)
int bin_reduce_obs(lbm_bin_ctx *c, const double *rho, const double *vel, double *out)
{
    const int nb = nred_blocks(c->n);
    double *part = bws(c, c->o_part), *res = bws(c, c->o_res);
    reduce_obs_kernel<<<nb, RED_THREADS, 0, c->stream>>>(c->n, 0.0, rho, vel, nullptr, part);
    finish_kernel<<<1, RED_THREADS, 0, c->stream>>>(nb, OBS_NV, OBS_OPS, part, res);
    if (hipGetLastError() != hipSuccess) return LBM_E_DEVICE;
    if (hipMemcpyAsync(out, res, OBS_NV * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return LBM_E_DEVICE;
    return hipStreamSynchronize(c->stream) == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

// per-direction sums of one stored distribution into h[Q]
template <class L> int bin_pop_sums(lbm_bin_ctx *c, const double *src, double *h)
{
    const int nb = nred_blocks(c->n);
    double *part = bws(c, c->o_part), *res = bws(c, c->o_res);
    reduce_pops_kernel<L, double><<<nb, RED_THREADS, 0, c->stream>>>(bin_geom(c), src, part);
    finish_kernel<<<1, RED_THREADS, 0, c->stream>>>(nb, L::Q, 0ull, part, res);
    if (hipGetLastError() != hipSuccess) return LBM_E_DEVICE;
    if (hipMemcpyAsync(h, res, L::Q * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return LBM_E_DEVICE;
    return hipStreamSynchronize(c->stream) == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

template <class L> int bin_totals_t(lbm_bin_ctx *c, double *mass, double *phi_total, double *mom)
{
    double hf[19], hg[19];
    // Every stored entry is read once per step, so its per-direction sums
    // give the totals; with walls a bounced entry arrives reversed, so the
    // state is first streamed into the idle buffers (free between steps).
    const double *fs = bin_f(c, c->cur), *gs = bin_g(c, c->cur);
    if (c->p.wall) {
        bin_state_kernel<L><<<grid1(c->n), 256, 0, c->stream>>>(bin_geom(c), true, true, fs, bin_f(c, c->cur ^ 1));
        bin_state_kernel<L><<<grid1(c->n), 256, 0, c->stream>>>(bin_geom(c), true, true, gs, bin_g(c, c->cur ^ 1));
        fs = bin_f(c, c->cur ^ 1);
        gs = bin_g(c, c->cur ^ 1);
    }
    int rc = bin_pop_sums<L>(c, fs, hf);
    if (rc == LBM_OK) rc = bin_pop_sums<L>(c, gs, hg);
    if (rc != LBM_OK) return rc;
    double m = 0, ph = 0, mx = 0, my = 0, mz = 0;
    for (int i = 0; i < L::Q; i++) {
        m += hf[i];
        ph += hg[i];
        mx += L::ex[i] * hf[i];
        my += L::ey[i] * hf[i];
        mz += L::ez[i] * hf[i];
    }
    if (mass) *mass = m;
    if (phi_total) *phi_total = ph;
    if (mom) {
        mom[0] = mx;
        mom[1] = my;
        mom[2] = mz;
    }
    return LBM_OK;
}

template <class L> void bin_state_io_t(lbm_bin_ctx *c, double *fo, double *go, const double *fi, const double *gi)
{
    const bool w = c->p.wall != 0;
    if (fo) {
        bin_state_kernel<L><<<grid1(c->n), 256, 0, c->stream>>>(bin_geom(c), w, true, bin_f(c, c->cur), fo);
        bin_state_kernel<L><<<grid1(c->n), 256, 0, c->stream>>>(bin_geom(c), w, true, bin_g(c, c->cur), go);
    } else {
        bin_state_kernel<L><<<grid1(c->n), 256, 0, c->stream>>>(bin_geom(c), w, false, fi, bin_f(c, c->cur));
        bin_state_kernel<L><<<grid1(c->n), 256, 0, c->stream>>>(bin_geom(c), w, false, gi, bin_g(c, c->cur));
    }
}

} // namespace

extern "C" {

void lbm_bin_params_default(lbm_bin_params *p)
{
    if (!p) return;
    p->phi_a = -0.02;
    p->phi_b = 0.02;
    p->kappa = 0.04;
    p->gamma = 1.0;
    p->tau = 1.0;
    p->tau_phi = 1.0;
    p->lattice = LBM_D2Q9;
    p->nx = 100;
    p->ny = 100;
    p->nz = 1;
    p->wall = 0;
    p->scheme = LBM_SCHEME_EQ;
    p->B = p->D = NAN;
    p->wp_diag = p->wt_diag = p->wxx_diag = NAN;
    p->tile = -1;
    p->planes_per_block = 0;
}

size_t lbm_bin_workspace_bytes(const lbm_bin_params *p)
{
    if (!bin_valid(p)) return 0;
    lbm_bin_ctx c{};
    c.p = *p;
    bin_layout(&c);
    return c.total;
}

int lbm_bin_init(lbm_bin_ctx **out, const lbm_bin_params *p, void *dev_workspace, size_t bytes,
                 void *stream, const double *dev_rho0, const double *dev_phi0, const double *dev_u0)
{
    if (!out || !bin_valid(p) || !dev_workspace || !dev_rho0 || !dev_phi0) return LBM_E_INVAL;
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN) return LBM_E_INVAL;
    lbm_bin_ctx *c = new (std::nothrow) lbm_bin_ctx();
    if (!c) return LBM_E_NOMEM;
    c->p = *p;
    bin_layout(c);
    if (bytes < c->total) {
        delete c;
        return LBM_E_NOMEM;
    }
    c->ws = static_cast<char *>(dev_workspace);
    c->stream = static_cast<hipStream_t>(stream);
    c->cur = 0;
    c->steps = 0;
    if (p->lattice == LBM_D2Q9) {
        c->nx = p->nx; c->ny = 1; c->np = p->ny;
    } else {
        c->nx = p->nx; c->ny = p->ny; c->np = p->nz;
    }
    c->n = (long long)p->nx * p->ny * p->nz;
    c->tile = p->tile >= 0 ? p->tile : (p->lattice == LBM_D2Q9 ? 0 : 3);
    c->cp = p->planes_per_block > 0 ? std::min(p->planes_per_block, c->np) : bin_default_planes(c, c->tile);
    c->c = bin_coefs(p);
    // the initial fields must be finite with rho > 0
    double obs[OBS_NV];
    int rc = bin_reduce_obs(c, dev_rho0, nullptr, obs);
    double obs_phi[OBS_NV];
    if (rc == LBM_OK) rc = bin_reduce_obs(c, dev_phi0, nullptr, obs_phi);
    if (rc != LBM_OK) {
        delete c;
        return rc;
    }
    // obs_phi[2] counts non-finite values and phi <= 0; only non-finite is bad
    if (obs[2] != 0.0 || !std::isfinite(obs_phi[5])) {
        delete c;
        return LBM_E_INVAL;
    }
    const bool force = p->scheme == LBM_SCHEME_FORCE;
    const Geom g = bin_geom(c);
    const unsigned nb = grid1(c->n);
    double *f0 = bin_f(c, 0), *g0 = bin_g(c, 0);
    bin_dispatch(p->lattice, [&](auto l) {
        using L = decltype(l);
        if (force) bin_init_kernel<L, true><<<nb, 256, 0, c->stream>>>(g, c->c, p->wall, dev_rho0, dev_phi0, dev_u0, f0, g0);
        else bin_init_kernel<L, false><<<nb, 256, 0, c->stream>>>(g, c->c, p->wall, dev_rho0, dev_phi0, dev_u0, f0, g0);
    });
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        delete c;
        return LBM_E_DEVICE;
    }
    *out = c;
    return LBM_OK;
}

int lbm_bin_step(lbm_bin_ctx *c, long long nsteps)
{
    if (!c || nsteps < 0) return LBM_E_INVAL;
    for (long long s = 0; s < nsteps; s++) {
        bin_launch_step(c);
        c->cur ^= 1;
        c->steps++;
    }
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_bin_moments(lbm_bin_ctx *c, double *dev_rho, double *dev_phi, double *dev_vel, double *dev_mu)
{
    if (!c) return LBM_E_INVAL;
    double *ph = dev_phi ? dev_phi : (dev_mu ? bws(c, c->o_phi) : nullptr);
    bin_launch_moments(c, dev_rho, ph, dev_vel);
    if (dev_mu) {
        bin_dispatch(c->p.lattice, [&](auto l) {
            bin_mu_kernel<decltype(l)><<<grid1(c->n), 256, 0, c->stream>>>(bin_geom(c), c->c, c->p.wall, ph, dev_mu);
        });
    }
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_bin_max_spurious_u(lbm_bin_ctx *c, double *host_out)
{
    if (!c || !host_out) return LBM_E_INVAL;
    double *r = bws(c, c->o_rho), *v = bws(c, c->o_vel);
    bin_launch_moments(c, r, nullptr, v);
    if (hipGetLastError() != hipSuccess) return LBM_E_DEVICE;
    double obs[OBS_NV];
    int rc = bin_reduce_obs(c, r, v, obs);
    if (rc != LBM_OK) return rc;
    *host_out = obs[0];
    return obs[2] != 0.0 ? LBM_E_NONFINITE : LBM_OK;
}

int lbm_bin_invariants(lbm_bin_ctx *c, double *host_mass, double *host_phi, double *host_mom)
{
    if (!c) return LBM_E_INVAL;
    int rc = LBM_OK;
    bin_dispatch(c->p.lattice, [&](auto l) { rc = bin_totals_t<decltype(l)>(c, host_mass, host_phi, host_mom); });
    return rc;
}

int lbm_bin_get_state(lbm_bin_ctx *c, double *dev_f, double *dev_g)
{
    if (!c || !dev_f || !dev_g) return LBM_E_INVAL;
    bin_dispatch(c->p.lattice, [&](auto l) { bin_state_io_t<decltype(l)>(c, dev_f, dev_g, nullptr, nullptr); });
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_bin_set_state(lbm_bin_ctx *c, const double *dev_f, const double *dev_g)
{
    if (!c || !dev_f || !dev_g) return LBM_E_INVAL;
    bin_dispatch(c->p.lattice, [&](auto l) { bin_state_io_t<decltype(l)>(c, nullptr, nullptr, dev_f, dev_g); });
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

long long lbm_bin_steps_done(const lbm_bin_ctx *c) { return c ? c->steps : -1; }

int lbm_bin_tile_count(int lattice)
{
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19 && lattice != LBM_D3Q15) return LBM_E_INVAL;
    return bin_tile_count(lattice);
}

int lbm_bin_tile_shape(int lattice, int k, int *tile_x, int *tile_y)
{
    const int nt = lbm_bin_tile_count(lattice);
    if (nt < 0 || k < 0 || k >= nt || !tile_x || !tile_y) return LBM_E_INVAL;
    const TileShape t = bin_tile(lattice, k);
    *tile_x = t.tx;
    *tile_y = t.ty;
    return LBM_OK;
}

int lbm_bin_set_launch(lbm_bin_ctx *c, int tile, int planes)
{
    if (!c || tile >= bin_tile_count(c->p.lattice)) return LBM_E_INVAL;
    if (tile >= 0) c->tile = tile;
    if (planes > 0) c->cp = std::min(planes, c->np);
    return LBM_OK;
}

int lbm_bin_get_launch(const lbm_bin_ctx *c, int *tile, int *planes, int *workgroups)
{
    if (!c) return LBM_E_INVAL;
    if (tile) *tile = c->tile;
    if (planes) *planes = c->cp;
    if (workgroups) {
        int a, b, ch;
        bin_grid(c, c->tile, c->cp, a, b, ch);
        *workgroups = a * b * ch;
    }
    return LBM_OK;
}

int lbm_bin_destroy(lbm_bin_ctx *c)
{
    delete c;
    return LBM_OK;
}

} // extern "C"
