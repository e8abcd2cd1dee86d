// lbm_step.h -- the fused free-energy LBM step: pull-stream, moments,
// stencils, equilibrium (or body force), BGK collision, store.
//
// Storage: S[i][p][y][x] (SoA, x fastest) holds the post-collision population
// of direction i at its source site, so the post-streaming population of
// Eq. (latbolt) at r is S[i][r - e_i] ("pull").  FP64 storage keeps f_i; FP32
// storage keeps delta_i = f_i - s_i with a fixed per-direction shift s_i.
//
// One workgroup owns a TX x TY tile of a plane and marches through `cp`
// consecutive planes (D2Q9: rows along y, TY = 1; D3Q19: xy-planes along z).
// Density planes of the tile plus an H-site halo (H = 1 for the equilibrium
// scheme, H = 2 for the forcing scheme, whose force needs gradients one site
// beyond the tile) live in an LDS ring; for the forcing scheme a second ring
// holds the gradient of rho on the tile plus one site.  Each thread keeps the
// pulled populations of its own site in registers from the plane where they
// are loaded (H planes ahead) until that plane is collided.  Halo densities
// are recomputed from populations owned by neighbouring tiles (they come from
// L2 / MALL when the neighbours run concurrently, which the XCD-aware block
// order encourages).
#pragma once

#include "lbm_lattice.h"

namespace lbm {

template <class R> struct StepArgs {
    const void *src;
    void *dst;
    double *obs_rho;   // observation outputs (observe != 0)
    double *obs_vel;   // [3][n]
    int nx, ny, np;    // in-plane x, in-plane y (1 for D2Q9), number of planes
    long long n;       // sites
    int cp;            // planes per workgroup
    int tiles_x, tiles_y, chunks;
    int write_pops;    // store the collided populations into dst
    int observe;       // write rho and the velocity of the pre-step state
    Coefs<R> c;
};

template <class S, class R> __device__ __forceinline__ R ld(const S *p, long long k)
{
    return R(p[k]);
}

template <class L, int SCHEME, class S, class R, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void step_kernel(StepArgs<R> A)
{
    constexpr int Q = L::Q;
    constexpr bool FORCE = SCHEME == SCHEME_FORCE;
    constexpr int H = FORCE ? 2 : 1;            // density halo
    constexpr int HY = L::DIM == 3 ? H : 0;     // in-plane y halo
    constexpr int TXH = TX + 2 * H, TYH = TY + 2 * HY;
    constexpr int PL = TXH * TYH;               // LDS sites per density plane
    constexpr int NR = FORCE ? 5 : 4;           // density ring depth
    constexpr int GY = L::DIM == 3 ? 1 : 0;     // gradient ring in-plane y halo
    constexpr int TXG = TX + 2, TYG = TY + 2 * GY;
    constexpr int GPL = TXG * TYG;
    constexpr int NT = TX * TY;
    constexpr int NHALO = 2 * HY * TXH + 2 * H * TY;

    __shared__ R rho_s[NR * PL];
    __shared__ R grad_s[FORCE ? 3 * 3 * GPL : 1];

    const S *__restrict__ src = static_cast<const S *>(A.src);
    S *__restrict__ dst = static_cast<S *>(A.dst);
    const Coefs<R> &c = A.c;
    const int nx = A.nx, ny = A.ny, np = A.np;
    const long long n = A.n;

    // XCD-aware order: consecutive workgroup ids go to different XCDs, so
    // give each XCD a contiguous run of tiles (neighbours share halos in L2).
    int nb = A.tiles_x * A.tiles_y * A.chunks;
    int b = blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int tile_x = b % A.tiles_x;
    const int tile_y = (b / A.tiles_x) % A.tiles_y;
    const int chunk = b / (A.tiles_x * A.tiles_y);
    const int x0 = tile_x * TX, y0 = tile_y * TY;
    const int p0 = chunk * A.cp;
    const int npl = min(A.cp, np - p0);
    if (npl <= 0) return;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    // this thread's site (wrapped; out-of-range threads still fill LDS)
    const int gx = wrapg(x0 + tx, nx);
    const int gy = L::DIM == 3 ? wrapg(y0 + ty, ny) : 0;
    const bool own = (x0 + tx < nx) && (L::DIM == 2 || y0 + ty < ny);

    // pulled populations of the own site: fr[k] holds plane (collide + k)
    R fr[H + 1][Q];

    // pull the Q populations arriving at (x, y, plane p) and return rho
    auto pull = [&](int x, int y, int p, R f[Q]) -> R {
        R s = R(0);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            int xs = wrap1(x - ox<L>(i), nx);
            int ys = L::DIM == 3 ? wrap1(y - oy<L>(i), ny) : 0;
            int ps = wrap1(p - op<L>(i), np);
            long long k = ((long long)ps * ny + ys) * nx + xs;
            f[i] = ld<S, R>(src, (long long)i * n + k);
            s += f[i];
        }
        return s + c.shift_sum;
    };

    auto rho_at = [&](int lp, int lx, int ly) -> R & {
        return rho_s[(lp % NR) * PL + ly * TXH + lx];
    };

    // density of local plane lp (global p0 - H + lp) on the tile + halo;
    // the own site's pulled populations go to f
    auto fill_rho = [&](int lp, R(&f)[Q]) {
        int p = wrapg(p0 - H + lp, np);
        rho_at(lp, tx + H, ty + HY) = pull(gx, gy, p, f);
        for (int k = tid; k < NHALO; k += NT) {
            int lx, ly;
            if (k < HY * TXH) {
                ly = k / TXH;
                lx = k % TXH;
            } else if (k < 2 * HY * TXH) {
                int kk = k - HY * TXH;
                ly = TY + HY + kk / TXH;
                lx = kk % TXH;
            } else {
                int kk = k - 2 * HY * TXH;
                int cc = kk % (2 * H);
                ly = HY + kk / (2 * H);
                lx = cc < H ? cc : TX + cc;
            }
            int hx = wrapg(x0 - H + lx, nx);
            int hy = L::DIM == 3 ? wrapg(y0 - HY + ly, ny) : 0;
            R g[Q];
            rho_at(lp, lx, ly) = pull(hx, hy, p, g);
        }
    };

    // gradient of rho on the tile + 1 ring of local plane lp (forcing only)
    auto grad_at = [&](int lp, int comp, int lx, int ly) -> R & {
        return grad_s[((lp % 3) * 3 + comp) * GPL + ly * TXG + lx];
    };
    auto fill_grad = [&](int lp) {
        for (int k = tid; k < GPL; k += NT) {
            int lx = k % TXG, ly = k / TXG;
            int rx = lx + (H - 1), ry = ly + (HY - GY);
            R d0 = R(0), d1 = R(0), d2 = R(0);
#pragma unroll
            for (int i = 1; i < Q; i++) {
                R r = rho_at(lp + op<L>(i), rx + ox<L>(i), ry + oy<L>(i));
                R cr = coef_grad<L>(c, i) * r;
                if (L::ex[i]) d0 += R(L::ex[i]) * cr;
                if (L::ey[i]) d1 += R(L::ey[i]) * cr;
                if (L::ez[i]) d2 += R(L::ez[i]) * cr;
            }
            grad_at(lp, 0, lx, ly) = d0;
            grad_at(lp, 1, lx, ly) = d1;
            grad_at(lp, 2, lx, ly) = d2;
        }
    };

    // prologue: densities of planes p0-H .. p0+H-1, gradients of p0-1, p0
    {
        R tmp[Q];
        for (int lp = 0; lp < H; lp++) fill_rho(lp, tmp);
    }
    fill_rho(H, fr[0]);
    if constexpr (H == 2) fill_rho(H + 1, fr[1]);
    __syncthreads();
    if (FORCE) {
        fill_grad(1);
        fill_grad(2);
    }

    for (int k = 0; k < npl; k++) {
        const int lc = H + k;  // local index of the plane collided now
        fill_rho(lc + H, fr[H]);
        __syncthreads();
        if (FORCE) {
            fill_grad(lc + 1);
            __syncthreads();
        }
        const int lx = tx + H, ly = ty + HY;
        R rho = rho_at(lc, lx, ly);
        R j[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (L::ex[i]) j[0] += R(L::ex[i]) * fr[0][i];
            if (L::ey[i]) j[1] += R(L::ey[i]) * fr[0][i];
            if (L::ez[i]) j[2] += R(L::ez[i]) * fr[0][i];
        }
        R d[3] = {R(0), R(0), R(0)};
        R lap = R(0);
#pragma unroll
        for (int i = 1; i < Q; i++) {
            R r = rho_at(lc + op<L>(i), lx + ox<L>(i), ly + oy<L>(i));
            lap += coef_lap<L>(c, i) * (r - rho);
            if (!FORCE) {
                R cr = coef_grad<L>(c, i) * r;
                if (L::ex[i]) d[0] += R(L::ex[i]) * cr;
                if (L::ey[i]) d[1] += R(L::ey[i]) * cr;
                if (L::ez[i]) d[2] += R(L::ez[i]) * cr;
            }
        }
        R g[3] = {R(0), R(0), R(0)};
        if (FORCE) {
            const int gx1 = tx + 1, gy1 = ty + GY;
            d[0] = grad_at(lc, 0, gx1, gy1);
            d[1] = grad_at(lc, 1, gx1, gy1);
            d[2] = grad_at(lc, 2, gx1, gy1);
            // g_a = -sum_i c_i kappa (dn_a (dn . e_i) - e_ia |dn|^2 / 2),
            // dn the gradient at r + e_i: the divergence of the kappa part
            // of the pressure tensor, Eq. (pt), with the force stencil
#pragma unroll
            for (int i = 1; i < Q; i++) {
                int lp = lc + op<L>(i), qx = gx1 + ox<L>(i), qy = gy1 + oy<L>(i);
                R n0 = grad_at(lp, 0, qx, qy), n1 = grad_at(lp, 1, qx, qy),
                  n2 = grad_at(lp, 2, qx, qy);
                R de = R(L::ex[i]) * n0 + R(L::ey[i]) * n1 + R(L::ez[i]) * n2;
                R dd = R(0.5) * (n0 * n0 + n1 * n1 + n2 * n2);
                R cf = coef_force<L>(c, i);
                g[0] += cf * (n0 * de - R(L::ex[i]) * dd);
                g[1] += cf * (n1 * de - R(L::ey[i]) * dd);
                if (L::DIM == 3) g[2] += cf * (n2 * de - R(L::ez[i]) * dd);
            }
            g[0] *= -c.kappa;
            g[1] *= -c.kappa;
            g[2] *= -c.kappa;
        }
        R feq[Q];
        equilibrium<L, !FORCE>(c, rho, j, d, lap, feq);
        R F[Q];
        R inv_rho = R(1) / rho;
        R u[3] = {j[0] * inv_rho, j[1] * inv_rho, j[2] * inv_rho};
        if (FORCE) forcing<L>(c, u, g, F);
        const int p = wrapg(p0 + k, np);
        const long long site = ((long long)p * ny + gy) * nx + gx;
        if (own && A.write_pops) {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                R dlt = fr[0][i];
                R out = dlt + c.omega * (feq[i] - c.shift[i] - dlt);
                if (FORCE) out += F[i];
                dst[(long long)i * n + site] = S(out);
            }
        }
        if (own && A.observe) {
            A.obs_rho[site] = double(rho);
            R h = FORCE ? R(0.5) * inv_rho : R(0);
            A.obs_vel[site] = double(u[0] + h * g[0]);
            A.obs_vel[n + site] = double(u[1] + h * g[1]);
            A.obs_vel[2 * n + site] = double(L::DIM == 3 ? u[2] + h * g[2] : R(0));
        }
        // rotate the register ring
#pragma unroll
        for (int s = 0; s < H; s++)
#pragma unroll
            for (int i = 0; i < Q; i++) fr[s][i] = fr[s + 1][i];
        // No barrier here: the next density fill writes ring slot of plane
        // lc+H+1, which no thread reads in this iteration (ring depths 4 and
        // 5); the next gradient fill overwrites a plane read above only after
        // the next barrier.
    }
}

} // namespace lbm
