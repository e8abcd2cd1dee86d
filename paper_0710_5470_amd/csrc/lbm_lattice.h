// lbm_lattice.h -- lattice constants and per-site physics shared by the HIP
// kernels of this library (device side only).
//
// Velocity sets follow the paper's numbering (Section "Model" for D2Q9,
// Section "Extension to 3D" for D3Q19) because populations cross the C ABI
// in that order.  Weight classes are derived from the geometry of each
// velocity (axis/face vs diagonal/edge, which axes it touches), which
// reproduces the optimum tables of the paper's summary (2D) and Eq. (3dres)
// (3D, with w_1-6 = 1/6 and the axial w^aa = 5/12; the printed 1/3 values
// violate the second-moment condition of Appendix A).
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

enum Scheme { SCHEME_EQ = 0, SCHEME_FORCE = 1 };

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int DIM = 2;
    // components (x, y, z)
    static constexpr int ex[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
    static constexpr int ey[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int DIM = 3;
    static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
};

// Kernels march plane by plane: D2Q9 treats x as the in-plane axis and y as
// the marching axis; D3Q19 has an (x, y) plane and marches along z.  These
// give the in-plane offsets (ox, oy) and the plane offset (op) of velocity i.
template <class L> __host__ __device__ constexpr int ox(int i) { return L::ex[i]; }
template <class L> __host__ __device__ constexpr int oy(int i) { return L::DIM == 3 ? L::ey[i] : 0; }
template <class L> __host__ __device__ constexpr int op(int i) { return L::DIM == 3 ? L::ez[i] : L::ey[i]; }
template <class L> __host__ __device__ constexpr int nnz(int i)
{
    return (L::ex[i] != 0) + (L::ey[i] != 0) + (L::ez[i] != 0);
}
template <class L> __host__ __device__ constexpr int ecomp(int i, int a)
{
    return a == 0 ? L::ex[i] : (a == 1 ? L::ey[i] : L::ez[i]);
}

// Runtime coefficients of one problem (host fills them; see lbm_capi.hip).
template <class R> struct Coefs {
    R A, B;            // gradient stencil: on-axis, off-axis
    R C, D;            // Laplacian stencil: on-axis, off-axis (centre = -sum)
    R Ef, Ff;          // force-stencil: on-axis, off-axis
    R w_ax, w_off;     // velocity weights
    R wp_ax, wp_off;   // w^p
    R wt_ax, wt_off;   // w^t
    // w^aa: velocity along a (axis), axis velocity not along a,
    // off-axis velocity touching a, off-axis velocity not touching a (3D)
    R wm_para, wm_perp, wm_in, wm_out;
    R kappa;
    R omega;           // 1 / tau
    int lambda_on;
    // Always FP64: the van der Waals pressure is a small difference of two
    // large terms near coexistence (rho T/(1 - b rho) ~ a rho^2 ~ 4 in the
    // liquid), so it, c_s^2 and the static part of each equilibrium
    // population are evaluated in FP64 whatever R is.
    double a, b, T;
    double nu;         // (tau - 1/2) / 3, Eq. (viscous)
    double wp_ax_d, wp_off_d;
    double shift[19];  // FP32 storage shift s_i (0 for FP64 storage)
    double shift_sum;  // sum_i s_i
};

template <class L, class R> __device__ __forceinline__ R coef_grad(const Coefs<R> &c, int i)
{
    return nnz<L>(i) == 1 ? c.A : c.B;
}
template <class L, class R> __device__ __forceinline__ R coef_lap(const Coefs<R> &c, int i)
{
    return nnz<L>(i) == 1 ? c.C : c.D;
}
template <class L, class R> __device__ __forceinline__ R coef_force(const Coefs<R> &c, int i)
{
    return nnz<L>(i) == 1 ? c.Ef : c.Ff;
}

// van der Waals bulk pressure, Eq. (p0), and c_s^2 = dp0/drho (FP64).
template <class R> __device__ __forceinline__ double vdw_p0(const Coefs<R> &c, double rho)
{
    return rho * c.T / (1.0 - c.b * rho) - c.a * rho * rho;
}
template <class R> __device__ __forceinline__ double vdw_cs2(const Coefs<R> &c, double rho)
{
    double d = 1.0 - c.b * rho;
    return c.T / (d * d) - 2.0 * c.a * rho;
}

// Equilibrium of Eq. (equilibrium) for i >= 1 and Eq. (feq0) for i = 0,
// returned as deviations from the storage shift: out_i = f_i^eq - s_i.
// rho_dev = rho - sum_i s_i (rho itself when s = 0); j: momentum;
// d: discrete gradient of rho; lap: discrete Laplacian.  The rest
// deviation is rho_dev - sum_{i>=1} out_i, so the shift never enters the
// mass balance.  WITH_M adds the kappa d_a rho d_b rho terms (equilibrium
// scheme only).  Returns rho.
template <class L, bool WITH_M, class R>
__device__ __forceinline__ R equilibrium(const Coefs<R> &c, R rho_dev, const R j[3], const R d[3],
                                         R lap, R feq[L::Q])
{
    constexpr int DIM = L::DIM;
    const double rho_d = double(rho_dev) + c.shift_sum;
    const R rho = R(rho_d);
    R inv_rho = R(1) / rho;
    R u[3] = {j[0] * inv_rho, j[1] * inv_rho, DIM == 3 ? j[2] * inv_rho : R(0)};
    const double p0 = vdw_p0(c, rho_d);
    R lam = c.lambda_on ? R(c.nu * (1.0 - 3.0 * vdw_cs2(c, rho_d))) : R(0);
    R ud = u[0] * d[0] + u[1] * d[1] + (DIM == 3 ? u[2] * d[2] : R(0));
    R uu = u[0] * u[0] + u[1] * u[1] + (DIM == 3 ? u[2] * u[2] : R(0));
    // trace of X_ab = rho u_a u_b + lam (u_a d_b + u_b d_a + delta_ab u.d)
    R trX = rho * uu + lam * R(2 + DIM) * ud;
    R klap = c.kappa * rho * lap;
    R M[3] = {c.kappa * d[0] * d[0], c.kappa * d[1] * d[1], DIM == 3 ? c.kappa * d[2] * d[2] : R(0)};
    R Mxy = c.kappa * d[0] * d[1];
    R Myz = DIM == 3 ? c.kappa * d[1] * d[2] : R(0);
    R Mzx = DIM == 3 ? c.kappa * d[2] * d[0] : R(0);
    R sum = R(0);
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const int e0 = L::ex[i], e1 = L::ey[i], e2 = L::ez[i];
        const bool axis = nnz<L>(i) == 1;
        R eu = R(e0) * u[0] + R(e1) * u[1] + R(e2) * u[2];
        R ed = R(e0) * d[0] + R(e1) * d[1] + R(e2) * d[2];
        R ej = R(e0) * j[0] + R(e1) * j[1] + R(e2) * j[2];
        R ee = R(nnz<L>(i));
        // sum_ab (e_a e_b - delta_ab / 3) X_ab
        R eXe = rho * eu * eu + lam * (R(2) * eu * ed + ee * ud);
        R w = axis ? c.w_ax : c.w_off;
        R v = w * (ej + R(1.5) * (eXe - trX * R(1.0 / 3.0)));
        // static part w^p_i p0 - s_i in FP64, then the gradient terms
        v += R((axis ? c.wp_ax_d : c.wp_off_d) * p0 - c.shift[i]);
        v -= (axis ? c.wt_ax : c.wt_off) * klap;
        if (WITH_M) {
            R m = R(0);
#pragma unroll
            for (int a = 0; a < DIM; a++) {
                const bool touches = ecomp<L>(i, a) != 0;
                R wa = axis ? (touches ? c.wm_para : c.wm_perp) : (touches ? c.wm_in : c.wm_out);
                m += wa * M[a];
            }
            // off-diagonal weights e_a e_b / 4 (constraint list after Eq. (fi))
            if (e0 * e1 != 0) m += R(0.25 * e0 * e1) * Mxy;
            if (e1 * e2 != 0) m += R(0.25 * e1 * e2) * Myz;
            if (e2 * e0 != 0) m += R(0.25 * e2 * e0) * Mzx;
            v += m;
        }
        feq[i] = v;
        sum += v;
    }
    feq[0] = rho_dev - sum;
    return rho;
}

// Forcing term of Section "Using a forcing method":
// F_i = w_i [e.g + (3/2)(e_a e_b - delta_ab/3)(u_a g_b + u_b g_a)], i >= 1,
// and F_0 = -sum_{i>=1} F_i (zero mass source).
template <class L, class R>
__device__ __forceinline__ void forcing(const Coefs<R> &c, const R u[3], const R g[3], R F[L::Q])
{
    R ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
    R sum = R(0);
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const int e0 = L::ex[i], e1 = L::ey[i], e2 = L::ez[i];
        R eu = R(e0) * u[0] + R(e1) * u[1] + R(e2) * u[2];
        R eg = R(e0) * g[0] + R(e1) * g[1] + R(e2) * g[2];
        R w = nnz<L>(i) == 1 ? c.w_ax : c.w_off;
        // (3/2)(2 (e.u)(e.g) - (2/3) u.g)
        R v = w * (eg + R(3) * eu * eg - ug);
        F[i] = v;
        sum += v;
    }
    F[0] = -sum;
}

__device__ __forceinline__ int wrap1(int v, int n)
{
    // v in [-1, n]
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

__device__ __forceinline__ int wrapg(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

} // namespace lbm
