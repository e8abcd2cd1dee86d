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
// e_i . v summed over the nonzero components of e_i only.  Under IEEE rules
// the compiler may not drop a product with a zero component (0 * inf is
// NaN), so the plain three-term form costs a multiply-add per zero
// component.  With at most two nonzero components of +-1 (D2Q9, D3Q19) the
// result is the single rounding of the full dot product.
template <class L, class R> __device__ __forceinline__ R edot(int i, const R v[3])
{
    R s = R(0);
    bool any = false;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int e = ecomp<L>(i, a);
        if (e == 0) continue;
        const R t = e > 0 ? v[a] : -v[a];
        s = any ? s + t : t;
        any = true;
    }
    return s;
}
// Start value of a sum that the compiler can fold into its first term:
// -0 + x is x for every x, whereas +0 + x is not when x is -0.
template <class R> __device__ __forceinline__ constexpr R sum0() { return R(-0.0); }

// the velocity opposite to e_i
template <class L> __host__ __device__ constexpr int opp(int i)
{
    for (int j = 0; j < L::Q; j++)
        if (L::ex[j] == -L::ex[i] && L::ey[j] == -L::ey[i] && L::ez[j] == -L::ez[i]) return j;
    return -1;
}
// the first velocity of the off-axis (diagonal / edge) weight class
template <class L> __host__ __device__ constexpr int first_off()
{
    for (int j = 1; j < L::Q; j++)
        if (nnz<L>(j) > 1) return j;
    return -1;
}

// Runtime coefficients of one problem (host fills them; see lbm_capi.hip).
template <class R> struct Coefs {
    R A, B;            // gradient stencil: on-axis, off-axis
    R C, D;            // Laplacian stencil: on-axis, off-axis (centre = -sum)
    R Ef, Ff;          // force-stencil: on-axis, off-axis
    R w_ax, w_off;     // velocity weights
    R ow_ax, ow_off;   // omega w_ax, omega w_off (odd part of the collision)
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

// van der Waals bulk pressure, Eq. (p0), and c_s^2 = dp0/drho (FP64), from
// one reciprocal of 1 - b rho.
template <class R> __device__ __forceinline__ void vdw(const Coefs<R> &c, double rho, double &p0, double &cs2)
{
    const double inv = 1.0 / (1.0 - c.b * rho);
    const double tinv = c.T * inv;
    p0 = rho * tinv - c.a * rho * rho;
    cs2 = tinv * inv - 2.0 * c.a * rho;
}

// Site quantities the equilibrium of Eq. (equilibrium) needs for every
// direction.  rho_dev = rho - sum_i s_i (rho itself when s = 0); j:
// momentum; d: discrete gradient of rho; lap: discrete Laplacian.
//
// Per direction the second-moment term is (3/2) w_i sum_ab (e_ia e_ib -
// delta_ab / 3) X_ab with X_ab = rho u_a u_b + lam (u_a d_b + u_b d_a +
// delta_ab u.d); its contraction with e_i e_i is
//   (e.u) (rho e.u + 2 lam e.d) + lam |e|^2 u.d,
// and the terms that depend on the direction only through its weight class
// (w^p_i p0 - s_i, the trace part, -w^t_i kappa rho lap) are summed once per
// class into stc.
template <class R> struct EqSite {
    R rho, u[3];
    R lam2;                 // 2 lam
    R lud[2];               // lam |e|^2 u.d for |e|^2 = 1, 2
    R stc[2];               // class terms, axis and off-axis
    R M[3], Mxy, Myz, Mzx;  // kappa d_a rho d_b rho (equilibrium scheme)
};

template <class L, bool WITH_M, class R>
__device__ __forceinline__ EqSite<R> eq_site(const Coefs<R> &c, double rho_dev, const R j[3], const R d[3], R lap,
                                             double scale = 1.0)
{
    constexpr int DIM = L::DIM;
    EqSite<R> s;
    const double rho_d = rho_dev + c.shift_sum;
    s.rho = R(rho_d);
    const R inv_rho = R(1) / s.rho;
    s.u[0] = j[0] * inv_rho;
    s.u[1] = j[1] * inv_rho;
    s.u[2] = DIM == 3 ? j[2] * inv_rho : R(0);
    double p0, cs2;
    vdw(c, rho_d, p0, cs2);
    const R lam = c.lambda_on ? R(c.nu * (1.0 - 3.0 * cs2)) : R(0);
    const R ud = s.u[0] * d[0] + s.u[1] * d[1] + (DIM == 3 ? s.u[2] * d[2] : R(0));
    const R uu = s.u[0] * s.u[0] + s.u[1] * s.u[1] + (DIM == 3 ? s.u[2] * s.u[2] : R(0));
    s.lam2 = R(2) * lam;
    s.lud[0] = lam * ud;
    s.lud[1] = R(2) * s.lud[0];
    // trace of X_ab over 3
    const R trX3 = (s.rho * uu + lam * R(2 + DIM) * ud) * R(1.0 / 3.0);
    const R klap = c.kappa * s.rho * lap;
    if (WITH_M) {
        s.M[0] = c.kappa * d[0] * d[0];
        s.M[1] = c.kappa * d[1] * d[1];
        s.M[2] = DIM == 3 ? c.kappa * d[2] * d[2] : R(0);
        s.Mxy = c.kappa * d[0] * d[1];
        s.Myz = DIM == 3 ? c.kappa * d[1] * d[2] : R(0);
        s.Mzx = DIM == 3 ? c.kappa * d[2] * d[0] : R(0);
    }
    // the static part w^p_i p0 - s_i in FP64 (the storage shift is the same
    // within a weight class), then the class terms, all times `scale` (the
    // collision passes omega), rounded once: in FP32 these class terms are
    // the largest part of every moving population's update, so one rounding
    // at their scale instead of three keeps the per-step error at the size
    // of the storage rounding
    const double st_ax = c.wp_ax_d * p0 - c.shift[1];
    const double st_off = c.wp_off_d * p0 - c.shift[first_off<L>()];
    s.stc[0] = R(scale * (st_ax - double(R(1.5) * c.w_ax * trX3 + c.wt_ax * klap)));
    s.stc[1] = R(scale * (st_off - double(R(1.5) * c.w_off * trX3 + c.wt_off * klap)));
    return s;
}

// sum_ab e_a e_b X_ab for velocity i, from eu = e.u and ed = e.d
template <class L, class R>
__device__ __forceinline__ R exe(const EqSite<R> &s, int i, R eu, R ed)
{
    return eu * (s.rho * eu + s.lam2 * ed) + s.lud[nnz<L>(i) - 1];
}

// kappa-gradient terms sum_ab w^ab_i kappa d_a rho d_b rho of velocity i
// (equilibrium scheme)
template <class L, class R>
__device__ __forceinline__ R m_terms(const Coefs<R> &c, const EqSite<R> &s, int i)
{
    const int e0 = L::ex[i], e1 = L::ey[i], e2 = L::ez[i];
    const bool axis = nnz<L>(i) == 1;
    R m = sum0<R>();
#pragma unroll
    for (int a = 0; a < L::DIM; a++) {
        const bool touches = ecomp<L>(i, a) != 0;
        R wa = axis ? (touches ? c.wm_para : c.wm_perp) : (touches ? c.wm_in : c.wm_out);
        m += wa * s.M[a];
    }
    // off-diagonal weights e_a e_b / 4 (constraint list after Eq. (fi))
    if (e0 * e1 != 0) m += R(0.25 * e0 * e1) * s.Mxy;
    if (e1 * e2 != 0) m += R(0.25 * e1 * e2) * s.Myz;
    if (e2 * e0 != 0) m += R(0.25 * e2 * e0) * s.Mzx;
    return m;
}

// Equilibrium of velocity i >= 1 split into the part even in e_i (second
// moment terms, static part, gradient terms) and the odd part w_i e_i.j:
// f_i^eq - s_i = even + odd and f_opp(i)^eq - s_opp(i) = even - odd.
template <class L, bool WITH_M, class R>
__device__ __forceinline__ void eq_pair(const Coefs<R> &c, const EqSite<R> &s, int i, const R j[3],
                                        const R d[3], R &even, R &odd)
{
    const bool axis = nnz<L>(i) == 1;
    const R w = axis ? c.w_ax : c.w_off;
    even = (R(1.5) * w) * exe<L>(s, i, edot<L>(i, s.u), edot<L>(i, d)) + s.stc[axis ? 0 : 1];
    if (WITH_M) even += m_terms<L>(c, s, i);
    odd = w * edot<L>(i, j);
}

// Equilibrium of Eq. (equilibrium) for i >= 1 and Eq. (feq0) for i = 0,
// returned as deviations from the storage shift: out_i = f_i^eq - s_i.  The
// rest deviation is rho_dev - sum_{i>=1} out_i, so the shift never enters
// the mass balance.  WITH_M adds the kappa d_a rho d_b rho terms
// (equilibrium scheme only).  Returns rho.
template <class L, bool WITH_M, class R>
__device__ __forceinline__ R equilibrium(const Coefs<R> &c, R rho_dev, const R j[3], const R d[3],
                                         R lap, R feq[L::Q])
{
    const EqSite<R> s = eq_site<L, WITH_M>(c, double(rho_dev), j, d, lap);
    // opposite velocities share the even terms: each pair is evaluated once
    R sum = R(0);
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        if (opp<L>(i) < i) continue;
        R even, odd;
        eq_pair<L, WITH_M>(c, s, i, j, d, even, odd);
        feq[i] = even + odd;
        feq[opp<L>(i)] = even - odd;
        sum += even;
    }
    feq[0] = rho_dev - R(2) * sum;
    return s.rho;
}

// BGK collision of Eq. (latbolt) with the forcing term of section "Using a
// forcing method" when FORCE: out_i = f_i + omega (f_i^eq - f_i) + F_i for
// the populations fin (deviations from the shift).  Per pair of opposite
// velocities, with f^eq - s = even +- odd and F = fe +- fd (fe = w (3 (e.u)
// (e.g) - u.g), fd = w e.g):
//   E = omega even + fe,  D = omega odd + fd,
//   out_i = (1 - omega) f_i + (E + D),  out_opp = (1 - omega) f_opp + (E - D),
//   out_0 = (1 - omega) f_0 + omega rho_dev - 2 sum_pairs E
// (F_0 = -sum_{i>=1} F_i and f_0^eq = rho - sum_{i>=1} f_i^eq).  omega is
// folded into the per-class terms.  g: body force (FORCE only).  Returns the
// site quantities (rho, u) for the caller's observables.
// emit(i, v) receives each collided population as soon as it is final (the
// pair i, opp(i) together, the rest population last), so that callers can
// store it at once instead of keeping all Q values live.
template <class L, bool FORCE, class R, class Emit>
__device__ __forceinline__ EqSite<R> collide(const Coefs<R> &c, R rho_dev, const R j[3], const R d[3], R lap,
                                             const R g[3], const R fin[L::Q], Emit &&emit)
{
    // FP32: the moving populations' sum (small terms) and rho from it and
    // f_0 in FP64, for the pressure; the rest population then closes the
    // mass balance with a single rounding at its own scale (below).
    constexpr bool F32 = sizeof(R) == 4;
    R s_in = sum0<R>();
    if constexpr (F32) {
#pragma unroll
        for (int i = 1; i < L::Q; i++) s_in += fin[i];
    }
    const double rho_d = F32 ? double(s_in) + double(fin[0]) : double(rho_dev);
    const EqSite<R> s = eq_site<L, !FORCE>(c, rho_d, j, d, lap, double(c.omega));
    const R om = c.omega, keep = R(1) - c.omega;
    // per-class constant part of E: omega stc (scaled in eq_site) - w u.g
    R K[2] = {s.stc[0], s.stc[1]};
    if (FORCE) {
        const R ug = s.u[0] * g[0] + s.u[1] * g[1] + (L::DIM == 3 ? s.u[2] * g[2] : R(0));
        K[0] -= c.w_ax * ug;
        K[1] -= c.w_off * ug;
    }
    R sumE = sum0<R>();
    R s_out = sum0<R>();
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        if (opp<L>(i) < i) continue;
        const int o = opp<L>(i);
        const bool axis = nnz<L>(i) == 1;
        const R w = axis ? c.w_ax : c.w_off;
        const R eu = edot<L>(i, s.u);
        R E = (R(1.5) * om * w) * exe<L>(s, i, eu, edot<L>(i, d)) + K[axis ? 0 : 1];
        if (!FORCE) E += om * m_terms<L>(c, s, i);
        // FP32: omega w from the exact pairs (the first-moment identity then
        // holds exactly in FP32); FP64: formed here (one register pair fewer)
        R D = (F32 ? (axis ? c.ow_ax : c.ow_off) : om * w) * edot<L>(i, j);
        if (FORCE) {
            const R eg = edot<L>(i, g);
            E += (R(3) * w * eu) * eg;
            D += w * eg;
        }
        sumE += E;
        const R oi = keep * fin[i] + (E + D);
        const R oo = keep * fin[o] + (E - D);
        if constexpr (F32) {
            s_out += oi;
            s_out += oo;
        }
        emit(i, oi);
        emit(o, oo);
    }
    if constexpr (F32) {
        // out_0 = rho - sum_{i>=1} out_i = f_0 + sum_{i>=1} (f_i - out_i):
        // the mass exchanged with the moving populations is formed from small
        // terms and added to f_0 with one rounding, so a site's mass changes
        // by that one rounding per step, as with FP64 arithmetic.  (The
        // direct form below rounds at the scale of f_0 ~ rho four times per
        // step; in FP32 the total mass then drifts about ten times faster.)
        emit(0, fin[0] + (s_in - s_out));
    } else {
        emit(0, keep * fin[0] + (om * rho_dev - R(2) * sumE));
    }
    return s;
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
