// lbm_binary.h -- fused time step of the binary-fluid free-energy model.
//
// The paper's Introduction states that its analysis applies equally to other
// multiphase systems such as binary fluids.  This is that carry-over for the
// symmetric binary fluid: an ideal-gas carrier density rho (c_s^2 = 1/3) and
// an order parameter phi with bulk free energy pa phi^2/2 + pb phi^4/4 and
// square-gradient term kappa |grad phi|^2 / 2.  Two distributions advance
// together:
//   f_i: the tuned equilibrium of Eq. (equilibrium)/(feq0) with phi in the
//        place of the differentiated density: bulk pressure p0 = rho/3 +
//        pa phi^2/2 + 3 pb phi^4/4 on the w^p weights, -w^t_i kappa phi
//        lap(phi), and the w^ab_i kappa d_a phi d_b phi terms; the lambda
//        term of Eq. (viscous) vanishes because c_s^2 = 1/3;
//   g_i: an order-parameter distribution whose equilibrium has moments phi,
//        phi u and gamma mu delta + phi u u, mu = pa phi + pb phi^3 -
//        kappa lap(phi); the gamma mu term rides on the w^p weights, the
//        velocity terms on w_i, and g_0 closes the zeroth moment.
// Gradients and Laplacians of phi use the isotropic stencils of Eqs.
// (xderiv), (laplace) and (laplacian3d); both distributions relax by BGK,
// Eq. (latbolt), with times tau and tau_phi.
//
// Forcing scheme (section "Using a forcing method", carried over): the f
// equilibrium drops the w^ab terms and f receives the forcing terms of the
// body force g = -div(kappa d phi d phi - delta kappa |d phi|^2 / 2); phi is
// advected by v = u + g / (2 rho).  A step is the phi kernel, then one march
// (bin_force_step_kernel) that forms the gradient and the force in LDS.
//
// Storage is FP64 in the pull layout of the liquid-gas kernels: S[i][r]
// holds the post-collision population of direction i at its source site,
// and the population arriving at r is S[i][r - e_i].
//
// Walls (optional; the paper defines none): two walls halfway between
// planes at both ends of the marching axis (y for D2Q9, z for D3Q19), the
// other axes periodic.  A population whose source r - e_i lies beyond a wall
// is the one that left r towards the wall, reversed (halfway bounce-back):
// in the pull layout it is read from S[opp(i)][r], an entry no other site
// reads.  The stencils read a plane beyond a wall as its mirror image in the
// fluid (zero normal derivative of phi: a neutral wall); in the forcing
// scheme the force stencil reads, beyond a wall, the gradient of that
// mirrored field.
//
// March.  A workgroup owns an in-plane tile of TX x TY sites (TY = 1 for
// D2Q9, whose "planes" are rows) and a chunk of consecutive planes.  Per
// plane it (1) forms phi = sum_i g_i of the plane ahead, for the tile and a
// one-site in-plane halo, into an LDS ring of four planes, then (2) after
// one barrier collides the current plane: the stencils read the ring, the
// own-site f_i are pulled, the own-site g_i are the ones the thread summed
// for phi one plane earlier (kept in registers), and the collided values are
// stored at the site itself, aligned.  With four ring slots the plane being
// formed is never one still being read, so one barrier per plane suffices.
#pragma once

#include "lbm_aux.h"

namespace lbm {

// D3Q15, for the lattice comparison of section "Extension to 3D" (binary
// stepper only): the faces e1..e6 as in D3Q19, then the eight cube corners
// in opposite pairs.  The paper gives no D3Q15 tables; the host builds them
// as the paper builds D3Q19 (moments of Appendix A, isotropic leading
// error where a choice remains, free corner weights overridable).
struct D3Q15 {
    static constexpr int Q = 15;
    static constexpr int DIM = 3;
    static constexpr int ex[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
    static constexpr int ey[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
    static constexpr int ez[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};
};

// weight of the off-diagonal kappa d_a d_b terms: e_a e_b / 4 on the D2Q9
// diagonals and D3Q19 edges (the constraint list after Eq. (fi)), e_a e_b / 8
// on the D3Q15 corners (eight of them carry each pair a, b)
template <class L> __host__ __device__ constexpr double bin_wxy() { return L::Q == 15 ? 0.125 : 0.25; }

struct BinCoefs {
    double A, B;                 // gradient stencil: on-axis, off-axis
    double C, D;                 // Laplacian stencil: on-axis, off-axis
    double w_ax, w_off;          // velocity weights
    double wp_ax, wp_off;        // w^p
    double wt_ax, wt_off;        // w^t
    double wm_para, wm_perp, wm_in, wm_out;  // w^aa classes (as Coefs)
    double kappa;
    double omega, omega_g;       // 1 / tau, 1 / tau_phi
    double pa, pb;               // bulk free energy pa phi^2/2 + pb phi^4/4
    double gamma;                // mobility coefficient of the mu term
    double Ef, Ff;               // force stencil: on-axis, off-axis
};

struct BinArgs {
    BinCoefs c;
    const double *__restrict__ fsrc;
    const double *__restrict__ gsrc;
    double *__restrict__ fdst;
    double *__restrict__ gdst;
    int nx, ny, np;              // in-plane x, in-plane y (1 for D2Q9), planes
    long long stride;            // elements between direction arrays
    int tiles_x, tiles_y, cp;    // tiles per in-plane axis, planes per workgroup
    const double *__restrict__ phi;    // forcing scheme: phi field [n] of the state
};

template <class L> __device__ __forceinline__ double bin_grad_coef(const BinCoefs &c, int i)
{
    return nnz<L>(i) == 1 ? c.A : c.B;
}
template <class L> __device__ __forceinline__ double bin_lap_coef(const BinCoefs &c, int i)
{
    return nnz<L>(i) == 1 ? c.C : c.D;
}

// sum_ab w^ab_i kappa d_a phi d_b phi of velocity i; M[0..2] diagonal,
// M[3..5] = xy, yz, zx
template <class L> __device__ __forceinline__ double bin_m_terms(const BinCoefs &c, const double M[6], int i)
{
    const bool axis = nnz<L>(i) == 1;
    double m = 0.0;
#pragma unroll
    for (int a = 0; a < L::DIM; a++) {
        const bool touches = ecomp<L>(i, a) != 0;
        m += (axis ? (touches ? c.wm_para : c.wm_perp) : (touches ? c.wm_in : c.wm_out)) * M[a];
    }
    const int e0 = L::ex[i], e1 = L::ey[i], e2 = L::ez[i];
    if (e0 * e1 != 0) m += (bin_wxy<L>() * e0 * e1) * M[3];
    if (e1 * e2 != 0) m += (bin_wxy<L>() * e1 * e2) * M[4];
    if (e2 * e0 != 0) m += (bin_wxy<L>() * e2 * e0) * M[5];
    return m;
}

// Site quantities both collisions need.
struct BinSite {
    double rho, u[3], uu, phi, mu;
};

// Collide f at one site.  fin: populations arriving at the site; phi: the
// order parameter there (the sum of the arriving g, formed by the caller in
// the same order as the stencil's field); d, lap: gradient and Laplacian of
// phi.  emit(i, v) receives each collided value.  Returns what the g
// collision needs.  FORCE (the forcing scheme): no w^ab terms in the
// equilibrium; the body force gf enters through F_i = w_i (e.g + (3/2)
// (e e - delta/3) : (u g + g u)), F_0 = -sum F_i, per pair of opposite
// velocities fe = w (3 (e.u)(e.g) - u.g) and fd = w e.g; the returned
// velocity (which advects phi) is v = u + g / (2 rho).
template <class L, bool FORCE = false, class EF>
__device__ __forceinline__ BinSite bin_collide_f(const BinCoefs &c, const double fin[L::Q], double phi,
                                                 const double d[3], double lap, EF &&emit,
                                                 const double *gf = nullptr)
{
    constexpr int Q = L::Q, DIM = L::DIM;
    BinSite s;
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; i++) {
        rho += fin[i];
        if (L::ex[i]) j[0] += L::ex[i] * fin[i];
        if (L::ey[i]) j[1] += L::ey[i] * fin[i];
        if (L::ez[i]) j[2] += L::ez[i] * fin[i];
    }
    const double inv = 1.0 / rho;
    s.rho = rho;
    s.u[0] = j[0] * inv;
    s.u[1] = j[1] * inv;
    s.u[2] = DIM == 3 ? j[2] * inv : 0.0;
    s.uu = s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2];
    s.phi = phi;
    const double p2 = phi * phi;
    const double p0 = rho * (1.0 / 3.0) + 0.5 * c.pa * p2 + 0.75 * c.pb * p2 * p2;
    s.mu = c.pa * phi + c.pb * p2 * phi - c.kappa * lap;
    const double M[6] = {c.kappa * d[0] * d[0], c.kappa * d[1] * d[1], c.kappa * d[2] * d[2],
                         c.kappa * d[0] * d[1], c.kappa * d[1] * d[2], c.kappa * d[2] * d[0]};
    // per-class terms: w^p p0 - (3/2) w rho u^2 / 3 - w^t kappa phi lap
    const double trX3 = rho * s.uu * (1.0 / 3.0);
    const double klap = c.kappa * phi * lap;
    const double stc[2] = {c.wp_ax * p0 - 1.5 * c.w_ax * trX3 - c.wt_ax * klap,
                           c.wp_off * p0 - 1.5 * c.w_off * trX3 - c.wt_off * klap};
    const double om = c.omega, keep = 1.0 - om;
    double ug = 0.0;
    if (FORCE) ug = s.u[0] * gf[0] + s.u[1] * gf[1] + (DIM == 3 ? s.u[2] * gf[2] : 0.0);
    double sumE = 0.0, sumF = 0.0;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        if (opp<L>(i) < i) continue;
        const int o = opp<L>(i);
        const bool axis = nnz<L>(i) == 1;
        const double w = axis ? c.w_ax : c.w_off;
        const double eu = edot<L>(i, s.u);
        // even = (3/2) w rho (e.u)^2 + class terms + w^ab terms; odd = w e.j
        double even = 1.5 * w * rho * eu * eu + stc[axis ? 0 : 1];
        if (!FORCE) even += bin_m_terms<L>(c, M, i);
        const double odd = w * edot<L>(i, j);
        sumE += even;
        double fe = 0.0, fd = 0.0;
        if (FORCE) {
            const double eg = edot<L>(i, gf);
            fe = w * (3.0 * eu * eg - ug);
            fd = w * eg;
            sumF += fe;
        }
        emit(i, keep * fin[i] + om * (even + odd) + (fe + fd));
        emit(o, keep * fin[o] + om * (even - odd) + (fe - fd));
    }
    emit(0, keep * fin[0] + om * (rho - 2.0 * sumE) - 2.0 * sumF);
    if (FORCE) {
        const double h = 0.5 * inv;
        s.u[0] += gf[0] * h;
        s.u[1] += gf[1] * h;
        if (DIM == 3) s.u[2] += gf[2] * h;
        s.uu = s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2];
    }
    return s;
}

// Collide g at one site with the site quantities of the f collision.
template <class L, class EG>
__device__ __forceinline__ void bin_collide_g(const BinCoefs &c, const double gin[L::Q], const BinSite &s,
                                              EG &&emit)
{
    constexpr int Q = L::Q;
    // per-class terms: w^p gamma mu - (3/2) w phi u^2 / 3
    const double gmu = c.gamma * s.mu;
    const double gtc[2] = {c.wp_ax * gmu - 0.5 * c.w_ax * s.phi * s.uu,
                           c.wp_off * gmu - 0.5 * c.w_off * s.phi * s.uu};
    const double om = c.omega_g, keep = 1.0 - om;
    double sumG = 0.0;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        if (opp<L>(i) < i) continue;
        const int o = opp<L>(i);
        const bool axis = nnz<L>(i) == 1;
        const double w = axis ? c.w_ax : c.w_off;
        const double eu = edot<L>(i, s.u);
        // even = (3/2) w phi (e.u)^2 + class terms; odd = w phi e.u
        const double even = 1.5 * w * s.phi * eu * eu + gtc[axis ? 0 : 1];
        const double odd = w * s.phi * eu;
        sumG += even;
        emit(i, keep * gin[i] + om * (even + odd));
        emit(o, keep * gin[o] + om * (even - odd));
    }
    emit(0, keep * gin[0] + om * (s.phi - 2.0 * sumG));
}

// Wrapped coordinates of a column: value, value - 1, value + 1.
__device__ __forceinline__ void wrap3(int v, int n, int (&w)[3])
{
    const int a = wrapg(v, n);
    w[0] = a;
    w[1] = a == 0 ? n - 1 : a - 1;
    w[2] = a == n - 1 ? 0 : a + 1;
}
// the coordinate a population of offset o arrives from: x - o
__device__ __forceinline__ int from3(const int (&w)[3], int o) { return o > 0 ? w[1] : (o < 0 ? w[2] : w[0]); }

template <class L, int TX, int TY, bool WALL>
__global__ __launch_bounds__(TX * TY) void bin_step_kernel(BinArgs a)
{
    constexpr int Q = L::Q, NT = TX * TY;
    constexpr int HY = L::DIM == 3 ? 1 : 0;
    constexpr int PW = TX + 2, PH = TY + 2 * HY, PL = PW * PH;
    constexpr int NIT = (PL + NT - 1) / NT;
    __shared__ double ring[4][PL];

    const int tid = threadIdx.x;
    // Workgroup ids are dealt to the XCDs round-robin.  D2Q9: give each XCD
    // a contiguous run of rows instead, so the rows a workgroup's halo reads
    // are fetched under the same L2 (measured faster).  D3Q19 keeps the
    // round-robin order: the contiguous order fetches fewer bytes but runs
    // slower there.
    int b = blockIdx.x;
    if (L::DIM == 2 && (gridDim.x & 7) == 0) b = (b & 7) * (gridDim.x >> 3) + (b >> 3);
    const int bx = b % a.tiles_x;
    b /= a.tiles_x;
    const int by = b % a.tiles_y;
    const int ch = b / a.tiles_y;
    const int x0 = bx * TX, y0 = by * TY;
    const int p_begin = ch * a.cp;
    const int p_end = min(p_begin + a.cp, a.np);
    const long long nxy = (long long)a.nx * a.ny;

    // own site
    const int tx = tid % TX, ty = tid / TX;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < a.nx && y < a.ny;
    const int c_own = (ty + HY) * PW + tx + 1;
    // Ring entries this thread forms: its own site first (k = 0), so the g
    // it sums for phi of the plane ahead are the ones it collides there one
    // plane later, then halo entries h = tid + (k - 1) NT: the rows below
    // and above the tile (3D), then its left and right columns.
    constexpr int H = PL - NT;
    int rx[NIT][3], ry[NIT][3], re[NIT];
    bool rv[NIT];
#pragma unroll
    for (int k = 0; k < NIT; k++) {
        int lx, ly;
        if (k == 0) {
            lx = tx;
            ly = ty;
            rv[k] = true;
        } else {
            const int h = tid + (k - 1) * NT;
            rv[k] = h < H;
            if (L::DIM == 3 && h < 2 * PW) {
                lx = h % PW - 1;
                ly = h < PW ? -1 : TY;
            } else {
                const int h2 = L::DIM == 3 ? h - 2 * PW : h;
                lx = (h2 & 1) ? TX : -1;
                ly = h2 >> 1;
            }
        }
        re[k] = (ly + HY) * PW + lx + 1;
        wrap3(x0 + lx, a.nx, rx[k]);
        wrap3(y0 + ly, a.ny, ry[k]);
    }

    // Address of the population of direction i arriving at (X[0], Y[0], P[0]).
    // With walls, a direction whose source plane lies beyond a wall (the
    // same for the whole workgroup) reads the own site's opposite direction:
    // the choice is made on the 32-bit direction and coordinates, and one
    // address is formed from them.
    auto src_index = [&](const int (&X)[3], const int (&Y)[3], const int (&P)[3], int i) {
        if (WALL && op<L>(i) != 0) {
            const bool b = op<L>(i) > 0 ? P[0] == 0 : P[0] == a.np - 1;
            const int dir = b ? opp<L>(i) : i;
            const int xs = b ? X[0] : from3(X, ox<L>(i));
            const int ys = b ? Y[0] : from3(Y, oy<L>(i));
            const int ps = b ? P[0] : from3(P, op<L>(i));
            return (long long)dir * a.stride + (long long)ps * nxy + (long long)ys * a.nx + xs;
        }
        return (long long)i * a.stride + (long long)from3(P, op<L>(i)) * nxy +
               (long long)from3(Y, oy<L>(i)) * a.nx + from3(X, ox<L>(i));
    };
    // phi of plane p for every ring entry, into ring slot s; the own site's
    // arriving g into gown.  With walls a plane beyond a wall is the mirror
    // image of the one inside it.
    auto form_phi = [&](int p, int s, double (&gown)[Q]) {
        int P[3];
        if (WALL) p = p < 0 ? -1 - p : (p >= a.np ? 2 * a.np - 1 - p : p);
        wrap3(p, a.np, P);
#pragma unroll
        for (int k = 0; k < NIT; k++) {
            if (!rv[k]) continue;
            double v = 0.0;
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const double gi = a.gsrc[src_index(rx[k], ry[k], P, i)];
                if (k == 0) gown[i] = gi;
                v += gi;
            }
            ring[s][re[k]] = v;
        }
    };

    double gcur[Q], gnext[Q];
    form_phi(p_begin - 1, 0, gnext);
    form_phi(p_begin, 1, gcur);
    for (int t = 0; p_begin + t < p_end; t++) {
        form_phi(p_begin + t + 1, (t + 2) & 3, gnext);
        __syncthreads();
        if (own) {
            const int p = p_begin + t;
            const double *sl[3] = {ring[t & 3], ring[(t + 1) & 3], ring[(t + 2) & 3]};
            const double phi = sl[1][c_own];
            double d[3] = {0.0, 0.0, 0.0}, lap = 0.0;
#pragma unroll
            for (int i = 1; i < Q; i++) {
                const double v = sl[1 + op<L>(i)][c_own + oy<L>(i) * PW + ox<L>(i)];
                const double g = bin_grad_coef<L>(a.c, i) * v;
                if (L::ex[i]) d[0] += L::ex[i] * g;
                if (L::ey[i]) d[1] += L::ey[i] * g;
                if (L::ez[i]) d[2] += L::ez[i] * g;
                lap += bin_lap_coef<L>(a.c, i) * (v - phi);
            }
            int P[3];
            wrap3(p, a.np, P);
            const long long site = (long long)p * nxy + (long long)y * a.nx + x;
            double fin[Q];
#pragma unroll
            for (int i = 0; i < Q; i++) fin[i] = a.fsrc[src_index(rx[0], ry[0], P, i)];
            const BinSite st = bin_collide_f<L>(a.c, fin, phi, d, lap, [&](int i, double v) {
                __builtin_nontemporal_store(v, a.fdst + (long long)i * a.stride + site);
            });
            bin_collide_g<L>(a.c, gcur, st, [&](int i, double v) {
                __builtin_nontemporal_store(v, a.gdst + (long long)i * a.stride + site);
            });
        }
#pragma unroll
        for (int i = 0; i < Q; i++) gcur[i] = gnext[i];
    }
}

// Forcing scheme, fused: one march per step after the phi kernel.  Per
// plane: (1) the phi field of the plane two ahead, with a two-site in-plane
// halo, into an LDS ring of five planes; barrier; (2) the
// gradient of phi on the plane ahead, with a one-site halo, into a ring of
// three planes; barrier; (3) the collision of the current plane: phi and
// lap(phi) from the phi ring, the body force -sum_b d_b T_ab with the force
// stencil from the gradients of the neighbours (T_ab = kappa d_a phi d_b phi
// - delta_ab kappa |d phi|^2 / 2 formed at each), the own f and g pulled.  A
// plane is written into the phi ring only after every thread has left the
// collision that last read that slot (five slots, written before the first
// barrier), and into the gradient ring only after the first barrier of the
// next plane (three slots).  With walls the phi field is continued beyond a
// wall as its mirror image (to any depth: period 2n along the marching
// axis), so the gradient ring's planes beyond a wall are the mirrored
// field's gradients and the force stencil reads them there; populations
// whose source lies beyond a wall are bounced back.
template <class L, int TX, int TY, bool WALL>
__global__ __launch_bounds__(TX * TY) void bin_force_step_kernel(BinArgs a)
{
    constexpr int Q = L::Q, NT = TX * TY;
    constexpr int HY = L::DIM == 3 ? 1 : 0;
    constexpr int PW2 = TX + 4, PL2 = PW2 * (TY + 4 * HY);  // phi: two-site halo
    constexpr int PW1 = TX + 2, PL1 = PW1 * (TY + 2 * HY);  // gradient: one-site halo
    constexpr int N2 = (PL2 + NT - 1) / NT, N1 = (PL1 + NT - 1) / NT;
    __shared__ double phis[5][PL2];
    __shared__ double grd[3][3][PL1];

    const int tid = threadIdx.x;
    int b = blockIdx.x;
    if (L::DIM == 2 && (gridDim.x & 7) == 0) b = (b & 7) * (gridDim.x >> 3) + (b >> 3);
    const int bx = b % a.tiles_x;
    b /= a.tiles_x;
    const int by = b % a.tiles_y;
    const int ch = b / a.tiles_y;
    const int x0 = bx * TX, y0 = by * TY;
    const int p_begin = ch * a.cp;
    const int p_end = min(p_begin + a.cp, a.np);
    const long long nxy = (long long)a.nx * a.ny;

    const int tx = tid % TX, ty = tid / TX;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < a.nx && y < a.ny;
    int ox3[3], oy3[3];
    wrap3(x, a.nx, ox3);
    wrap3(y, a.ny, oy3);
    const int c2 = (ty + 2 * HY) * PW2 + tx + 2;  // own entry in the phi ring
    const int c1 = (ty + HY) * PW1 + tx + 1;      // own entry in the gradient ring

    // in-plane offsets of this thread's phi-ring entries
    int off2[N2];
#pragma unroll
    for (int k = 0; k < N2; k++) {
        const int e = tid + k * NT;
        const int wx = wrapg(x0 + e % PW2 - 2, a.nx);
        const int wy = wrapg(y0 + e / PW2 - 2 * HY, a.ny);
        off2[k] = e < PL2 ? wy * a.nx + wx : -1;
    }
    auto load_phi = [&](int p, int s) {
        int pr = wrapg(p, WALL ? 2 * a.np : a.np);
        if (WALL && pr >= a.np) pr = 2 * a.np - 1 - pr;
        const long long base = (long long)pr * nxy;
#pragma unroll
        for (int k = 0; k < N2; k++)
            if (off2[k] >= 0) phis[s][tid + k * NT] = a.phi[base + off2[k]];
    };
    // gradient of the plane in phi slot sc (neighbour planes in sm, sp)
    auto gradient = [&](int sm, int sc, int sp, int gs) {
        const double *sl[3] = {phis[sm], phis[sc], phis[sp]};
#pragma unroll
        for (int k = 0; k < N1; k++) {
            const int e = tid + k * NT;
            if (e >= PL1) continue;
            const int r2 = (e / PW1 + HY) * PW2 + e % PW1 + 1;  // the entry in phi-ring coordinates
            double d[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 1; i < Q; i++) {
                const double v = bin_grad_coef<L>(a.c, i) * sl[1 + op<L>(i)][r2 + oy<L>(i) * PW2 + ox<L>(i)];
                if (L::ex[i]) d[0] += L::ex[i] * v;
                if (L::ey[i]) d[1] += L::ey[i] * v;
                if (L::ez[i]) d[2] += L::ez[i] * v;
            }
            grd[gs][0][e] = d[0];
            grd[gs][1][e] = d[1];
            grd[gs][2][e] = d[2];
        }
    };
    // slots: phi of plane q at (q - p_begin + 2) % 5, gradient at (q - p_begin + 1) % 3
    load_phi(p_begin - 2, 0);
    load_phi(p_begin - 1, 1);
    load_phi(p_begin, 2);
    load_phi(p_begin + 1, 3);
    __syncthreads();
    gradient(0, 1, 2, 0);
    gradient(1, 2, 3, 1);
    for (int t = 0; p_begin + t < p_end; t++) {
        const int p = p_begin + t;
        load_phi(p + 2, (t + 4) % 5);
        __syncthreads();
        gradient((t + 2) % 5, (t + 3) % 5, (t + 4) % 5, (t + 2) % 3);
        __syncthreads();
        if (!own) continue;
        const double *sl[3] = {phis[(t + 1) % 5], phis[(t + 2) % 5], phis[(t + 3) % 5]};
        const int gsl[3] = {t % 3, (t + 1) % 3, (t + 2) % 3};
        const double phi = sl[1][c2];
        double lap = 0.0, gf[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 1; i < Q; i++) {
            lap += bin_lap_coef<L>(a.c, i) * (sl[1 + op<L>(i)][c2 + oy<L>(i) * PW2 + ox<L>(i)] - phi);
            // -sum_b (force stencil) e_ib T_ab at the neighbour r + e_i
            const int g = gsl[1 + op<L>(i)], e = c1 + oy<L>(i) * PW1 + ox<L>(i);
            const double d[3] = {grd[g][0][e], grd[g][1][e], L::DIM == 3 ? grd[g][2][e] : 0.0};
            const double h = 0.5 * a.c.kappa * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double k = nnz<L>(i) == 1 ? a.c.Ef : a.c.Ff;
#pragma unroll
            for (int bb = 0; bb < L::DIM; bb++) {
                const int eb = ecomp<L>(i, bb);
                if (eb == 0) continue;
#pragma unroll
                for (int aa = 0; aa < L::DIM; aa++)
                    gf[aa] -= (k * eb) * (a.c.kappa * d[aa] * d[bb] - (aa == bb ? h : 0.0));
            }
        }
        int P[3];
        wrap3(p, a.np, P);
        // source of direction i; beyond a wall the own site's opposite
        // direction (chosen on 32-bit values, one address formed)
        auto src = [&](int i) {
            if (WALL && op<L>(i) != 0) {
                const bool bb = op<L>(i) > 0 ? P[0] == 0 : P[0] == a.np - 1;
                const int dir = bb ? opp<L>(i) : i;
                const int xs = bb ? ox3[0] : from3(ox3, ox<L>(i));
                const int ys = bb ? oy3[0] : from3(oy3, oy<L>(i));
                const int ps = bb ? P[0] : from3(P, op<L>(i));
                return (long long)dir * a.stride + (long long)ps * nxy + (long long)ys * a.nx + xs;
            }
            return (long long)i * a.stride + (long long)from3(P, op<L>(i)) * nxy +
                   (long long)from3(oy3, oy<L>(i)) * a.nx + from3(ox3, ox<L>(i));
        };
        const long long site = (long long)p * nxy + (long long)y * a.nx + x;
        double fin[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) fin[i] = a.fsrc[src(i)];
        const double dz[3] = {0.0, 0.0, 0.0};  // no w^ab terms in this scheme
        const BinSite st = bin_collide_f<L, true>(a.c, fin, phi, dz, lap, [&](int i, double v) {
            __builtin_nontemporal_store(v, a.fdst + (long long)i * a.stride + site);
        }, gf);
        double gin[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) gin[i] = a.gsrc[src(i)];
        bin_collide_g<L>(a.c, gin, st, [&](int i, double v) {
            __builtin_nontemporal_store(v, a.gdst + (long long)i * a.stride + site);
        });
    }
}

// Pull-layout address of the population of direction i arriving at (x, y, p):
// S[i][r - e_i], or S[opp(i)][r] when r - e_i lies beyond a wall.
template <class L>
__device__ __forceinline__ long long bin_arrival(const Geom &g, bool wall, int x, int y, int p, int i)
{
    if (wall && op<L>(i) != 0) {
        const int ps = p - op<L>(i);
        if (ps < 0 || ps >= g.np) return (long long)opp<L>(i) * g.stride + site_index<L>(g, x, y, p);
    }
    return (long long)i * g.stride + neighbour<L>(g, x, y, p, i, -1);
}

// Site r + e_i read by a stencil; a plane beyond a wall is mirrored.
template <class L>
__device__ __forceinline__ long long bin_stencil_site(const Geom &g, bool wall, int x, int y, int p, int i)
{
    if (wall && op<L>(i) != 0) {
        const int pn = p + op<L>(i);
        if (pn < 0 || pn >= g.np) {
            const int xs = wrap1(x + ox<L>(i), g.nx);
            const int ys = L::DIM == 3 ? wrap1(y + oy<L>(i), g.ny) : 0;
            return site_index<L>(g, xs, ys, pn < 0 ? 0 : g.np - 1);
        }
    }
    return neighbour<L>(g, x, y, p, i, +1);
}

// f = f^eq(rho0, rho0 u0, phi0), g = g^eq(phi0, u0) with the stencils applied
// to phi0, stored in the pull layout (where each population is read).
template <class L, bool FORCE>
__global__ void bin_init_kernel(Geom g, BinCoefs c, bool wall, const double *__restrict__ rho0,
                                const double *__restrict__ phi0, const double *__restrict__ u0,
                                double *__restrict__ fdst, double *__restrict__ gdst)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
    const double phi = phi0[s], rho = rho0[s];
    double d[3] = {0, 0, 0}, lap = 0;
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const double v = phi0[bin_stencil_site<L>(g, wall, x, y, p, i)];
        const double cg = bin_grad_coef<L>(c, i) * v;
        d[0] += L::ex[i] * cg;
        d[1] += L::ey[i] * cg;
        d[2] += L::ez[i] * cg;
        lap += bin_lap_coef<L>(c, i) * (v - phi);
    }
    double u[3] = {0, 0, 0};
    if (u0) {
        u[0] = u0[s];
        u[1] = u0[g.stride + s];
        if (L::DIM == 3) u[2] = u0[2 * g.stride + s];
    }
    // equilibria = collision with omega = 1 of any populations with these
    // moments: feed the equilibrium moments through a rest-only input
    BinCoefs ce = c;
    ce.omega = 1.0;
    ce.omega_g = 1.0;
    double fin[L::Q], gin[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        fin[i] = 0.0;
        gin[i] = 0.0;
    }
    // populations carrying mass rho and momentum rho u: rest + one pair per axis
    fin[0] = rho;
    gin[0] = phi;
#pragma unroll
    for (int a = 0; a < L::DIM; a++) {
        // velocity +e_a is index 1 + 2a (paper numbering: axes first, +/- pairs)
        const double half = 0.5 * rho * u[a];
        fin[1 + 2 * a] += half;
        fin[2 + 2 * a] -= half;
    }
    // (the forcing scheme's equilibrium: no w^ab terms, no force at rest)
    const double zero[3] = {0.0, 0.0, 0.0};
    const BinSite st = bin_collide_f<L, FORCE>(ce, fin, phi, d, lap, [&](int i, double v) {
        fdst[bin_arrival<L>(g, wall, x, y, p, i)] = v;
    }, zero);
    bin_collide_g<L>(ce, gin, st, [&](int i, double v) {
        gdst[bin_arrival<L>(g, wall, x, y, p, i)] = v;
    });
}

// Observables of the pulled state: rho, phi, u = j / rho (for mu, a second
// pass applies the Laplacian to phi).
template <class L>
__global__ void bin_moments_kernel(Geom g, bool wall, const double *__restrict__ fsrc,
                                   const double *__restrict__ gsrc, const double *__restrict__ force,
                                   double *__restrict__ rho_out, double *__restrict__ phi_out,
                                   double *__restrict__ vel_out)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
    double rho = 0, phi = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const long long k = bin_arrival<L>(g, wall, x, y, p, i);
        const double v = fsrc[k];
        rho += v;
        phi += gsrc[k];
        j[0] += L::ex[i] * v;
        j[1] += L::ey[i] * v;
        j[2] += L::ez[i] * v;
    }
    if (rho_out) rho_out[s] = rho;
    if (phi_out) phi_out[s] = phi;
    if (vel_out) {  // u, plus g / (2 rho) for the forcing scheme
        double v[3] = {j[0] / rho, j[1] / rho, L::DIM == 3 ? j[2] / rho : 0.0};
        if (force)
            for (int a = 0; a < L::DIM; a++) v[a] += force[a * g.stride + s] / (2.0 * rho);
        vel_out[s] = v[0];
        vel_out[g.stride + s] = v[1];
        vel_out[2 * g.stride + s] = v[2];
    }
}

// Forcing scheme: the order parameter phi = sum_i g_i of the arriving
// populations (bounced back at walls), before each step and for
// observables ...
template <class L, bool WALL>
__global__ void bin_phi_kernel(Geom g, const double *__restrict__ gsrc, double *__restrict__ phi)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) v += gsrc[bin_arrival<L>(g, WALL, x, y, p, i)];
    phi[s] = v;
}

// ... and, for observables (the velocity v = u + g / (2 rho)), the gradient
// d phi with the gradient stencil (walls mirrored), dphi[3][n] ...
template <class L>
__global__ void bin_gradient_kernel(Geom g, BinCoefs c, bool wall, const double *__restrict__ phi,
                                    double *__restrict__ dphi)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
    double d[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const double v = bin_grad_coef<L>(c, i) * phi[bin_stencil_site<L>(g, wall, x, y, p, i)];
        if (L::ex[i]) d[0] += L::ex[i] * v;
        if (L::ey[i]) d[1] += L::ey[i] * v;
        if (L::ez[i]) d[2] += L::ez[i] * v;
    }
    dphi[s] = d[0];
    dphi[g.stride + s] = d[1];
    if (L::DIM == 3) dphi[2 * g.stride + s] = d[2];
}

// ... and the body force g_a = -sum_b d_b T_ab with the force stencil
// (section "Using a forcing method"), T_ab = kappa d_a phi d_b phi -
// delta_ab kappa |d phi|^2 / 2 formed at each neighbour from its gradient,
// force[3][n].  Beyond a wall the gradient is that of the mirror image: the
// mirror site's, its normal component reversed.
template <class L>
__global__ void bin_divergence_kernel(Geom g, BinCoefs c, bool wall, const double *__restrict__ dphi,
                                      double *__restrict__ force)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
    double f[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const long long nb = bin_stencil_site<L>(g, wall, x, y, p, i);
        double d[3] = {dphi[nb], dphi[g.stride + nb], L::DIM == 3 ? dphi[2 * g.stride + nb] : 0.0};
        if (wall && op<L>(i) != 0 && (p + op<L>(i) < 0 || p + op<L>(i) >= g.np)) d[L::DIM - 1] = -d[L::DIM - 1];
        const double h = 0.5 * c.kappa * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double k = nnz<L>(i) == 1 ? c.Ef : c.Ff;
#pragma unroll
        for (int b = 0; b < L::DIM; b++) {
            const int e = ecomp<L>(i, b);
            if (e == 0) continue;
            const double ke = k * e;
#pragma unroll
            for (int a = 0; a < L::DIM; a++) {
                const double T = c.kappa * d[a] * d[b] - (a == b ? h : 0.0);
                f[a] -= ke * T;
            }
        }
    }
    force[s] = f[0];
    force[g.stride + s] = f[1];
    force[2 * g.stride + s] = L::DIM == 3 ? f[2] : 0.0;
}

// mu = pa phi + pb phi^3 - kappa lap(phi) from a phi field
template <class L>
__global__ void bin_mu_kernel(Geom g, BinCoefs c, bool wall, const double *__restrict__ phi,
                              double *__restrict__ mu)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
    const double v0 = phi[s];
    double lap = 0;
#pragma unroll
    for (int i = 1; i < L::Q; i++) lap += bin_lap_coef<L>(c, i) * (phi[bin_stencil_site<L>(g, wall, x, y, p, i)] - v0);
    mu[s] = c.pa * v0 + c.pb * v0 * v0 * v0 - c.kappa * lap;
}

// Post-streaming populations out[i][r] (the populations arriving at r) from
// the pull layout, or (set) the reverse.
template <class L>
__global__ void bin_state_kernel(Geom g, bool wall, bool get, const double *__restrict__ in,
                                 double *__restrict__ out)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    int x, y, p;
    site_coords<L>(g, s, x, y, p);
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const long long k = bin_arrival<L>(g, wall, x, y, p, i);
        if (get) out[(long long)i * g.stride + s] = in[k];
        else out[k] = in[(long long)i * g.stride + s];
    }
}

} // namespace lbm
