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
// Densities (as rho - sum_i s_i) of the tile plus an H-site halo (H = 1 for
// the equilibrium scheme, below; H = 2 for the forcing scheme, lbm_force.h)
// live in an LDS ring of planes.  Each thread keeps the pulled populations
// of its own site in registers from the plane where they are loaded (H + 1
// planes ahead of the collision) until that plane is collided.  Halo
// densities are recomputed from populations owned by neighbouring tiles
// (they come from L2 / MALL when the neighbours run concurrently, which the
// XCD-aware workgroup order encourages).
//
// Population arrays are read and written through one buffer resource per
// array (32-bit byte offsets, hardware range check); the direction's offset
// rides in the scalar offset and the wrapped neighbour offsets are
// precomputed per thread, so a load needs no per-direction address work.
#pragma once

#include <type_traits>

#include "lbm_lattice.h"

namespace lbm {

template <class R> struct StepArgs {
    const void *src;
    void *dst;
    double *obs_rho;   // observation outputs (observe != 0)
    double *obs_vel;   // [3][n]
    int nx, ny, np;    // in-plane x, in-plane y (1 for D2Q9), number of planes
    long long n;       // sites; Q * n * sizeof(S) < 2^32 (checked by the host)
    int cp;            // planes per workgroup
    int tiles_x, tiles_y, chunks;
    int write_pops;    // store the collided populations into dst
    int observe;       // write rho and the velocity of the pre-step state
    Coefs<R> c;
};

// Raw buffer descriptor over `bytes` bytes from base (gfx9 family dword3:
// 32-bit data format, no swizzle).  One descriptor covers all directions of
// a population buffer; the direction offset rides in the scalar offset.
template <class S> __device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const S *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// FP32 arithmetic in the equilibrium marches with an FP64 density ring (see
// the ring in eq_tile)
#ifndef LBM_EQ_RING64
#define LBM_EQ_RING64 1
#endif
// Cache policy of the population stores: 2 sets the non-temporal bit (nt),
// so the stores stream past the caches instead of evicting the neighbour
// populations that halo loads re-read (the stored state is read again only
// in the next step, long after it has left the caches).
#ifndef LBM_STORE_CPOL
#define LBM_STORE_CPOL 2
#endif

__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff,
                                          LBM_STORE_CPOL);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(
                                              r, 0, 0, 0)), v),
                                          r, (int)voff, (int)soff, LBM_STORE_CPOL);
}

// Minimum waves per SIMD the step kernel is compiled for; 0 = per
// instance: four for the D2Q9 FP32 forcing kernel (its FP64 density ring
// takes it to 135 VGPRs, three waves; capped at 128 it keeps four, which
// this small, cache-resident kernel needs), the compiler's choice elsewhere.
#ifndef LBM_STEP_WAVES_PER_EU
#define LBM_STEP_WAVES_PER_EU 0
#endif
// The same for the batched (persistent) kernel; 0 = per instance: three
// waves per SIMD for the D2Q9 FP64 equilibrium kernel (172 -> 168 VGPRs,
// 4 dwords spilled; 2 % off the batched time-to-steady of 512 drops), the
// compiler's choice elsewhere (the larger kernels would spill heavily).
#ifndef LBM_BATCH_WAVES_PER_EU
#define LBM_BATCH_WAVES_PER_EU 0
#endif
template <class L, int SCHEME, class S, class R> constexpr int step_waves_per_eu()
{
    if (LBM_STEP_WAVES_PER_EU > 0) return LBM_STEP_WAVES_PER_EU;
    return (L::DIM == 2 && SCHEME == SCHEME_FORCE && sizeof(S) == 4 && sizeof(R) == 4) ? 4 : 1;
}
template <class L, int SCHEME, class S> constexpr int batch_waves_per_eu()
{
    if (LBM_BATCH_WAVES_PER_EU > 0) return LBM_BATCH_WAVES_PER_EU;
    return (L::DIM == 2 && SCHEME == SCHEME_EQ && sizeof(S) == 8) ? 3 : 1;
}

// One workgroup's share of a step: the tile at (x0, y0) of planes
// [p0, p0 + npl) of one problem.
template <class R> struct Job {
    const void *src;       // direction i of this problem at src + i * stride
    void *dst;
    long long stride;      // elements between direction arrays
    unsigned bytes;        // bytes addressable from src / dst (range check)
    double *obs_rho;       // [n]
    double *obs_vel;       // component a at obs_vel + a * obs_stride
    long long obs_stride;
    int nx, ny, np;        // in-plane x, in-plane y (1 for D2Q9), planes
    int x0, y0, p0, npl;
    int write_pops, observe;
};

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, not for its outstanding global loads.  (__syncthreads() is a
// workgroup-scope fence, which must also wait for direct-to-LDS loads, i.e.
// for the prefetch of the next planes.)  The memory clobber keeps the
// compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_sync()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The equilibrium scheme (Eq. (equilibrium)): gradients and Laplacian of
// the density are needed one site away, so the ring holds the tile plus a
// 1-site halo and the own populations stay in registers for H + 1 = 2
// planes after their density is stored.
template <class L, class S, class R, int TX, int TY>
__device__ __forceinline__ void eq_tile(const Job<R> &J, const Coefs<R> &c)
{
    constexpr int Q = L::Q;
    constexpr int H = 1;                        // density halo
    constexpr int HY = L::DIM == 3 ? H : 0;     // in-plane y halo
    constexpr int TXH = TX + 2 * H, TYH = TY + 2 * HY;
    constexpr int PL = TXH * TYH;               // LDS sites per density plane
    // density ring: planes lc - 1 .. lc + 2 are live; four slots, so a ring
    // slot is a mask, not a division
    constexpr int NR = 4;
    constexpr int NT = TX * TY;
    constexpr int NHALO = 2 * HY * TXH + 2 * H * TY;
    constexpr int NHT = (NHALO + NT - 1) / NT;  // halo sites per thread
    constexpr unsigned ES = sizeof(S);

    // FP32 arithmetic: densities in the ring as FP64 (the FP32 sum of the
    // moving deviations plus the rest one, not rounded at the scale of
    // rho - sum s_i), stencils on differences to the centre taken in FP64
    using RD = std::conditional_t<sizeof(R) == 4 && LBM_EQ_RING64, double, R>;
    __shared__ RD rho_s[NR * PL];

    const S *src = static_cast<const S *>(J.src);
    S *dst = static_cast<S *>(J.dst);
    const long long stride = J.stride;
    const int nx = J.nx, ny = J.ny, np = J.np;
    const int psz = nx * ny;  // elements per plane
    const int x0 = J.x0, y0 = J.y0, p0 = J.p0, npl = J.npl;
    const __amdgpu_buffer_rsrc_t rs = pop_rsrc(src, J.bytes);
    const __amdgpu_buffer_rsrc_t rd = pop_rsrc(dst, J.bytes);

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    // Own site (wrapped; threads past a ragged edge still fill LDS but do not
    // store).  X[k] / Y[k]: element offsets of x + k - 1 / y + k - 1.
    int X[3], Y[3];
    const int gx = wrapg(x0 + tx, nx);
    const int gy = L::DIM == 3 ? wrapg(y0 + ty, ny) : 0;
    X[0] = wrap1(gx - 1, nx); X[1] = gx; X[2] = wrap1(gx + 1, nx);
    if (L::DIM == 3) {
        Y[0] = wrap1(gy - 1, ny) * nx; Y[1] = gy * nx; Y[2] = wrap1(gy + 1, ny) * nx;
    } else {
        Y[0] = Y[1] = Y[2] = 0;
    }
    const bool own = (x0 + tx < nx) && (L::DIM == 2 || y0 + ty < ny);

    // Halo sites of this thread (fixed for the whole march).
    int hX[NHT][3], hY[NHT][3], hL[NHT];
    bool hv[NHT];
#pragma unroll
    for (int s = 0; s < NHT; s++) {
        const int k = tid + s * NT;
        hv[s] = k < NHALO;
        int lx = 0, ly = 0;
        if (k < HY * TXH) {
            ly = k / TXH;
            lx = k % TXH;
        } else if (k < 2 * HY * TXH) {
            const int kk = k - HY * TXH;
            ly = TY + HY + kk / TXH;
            lx = kk % TXH;
        } else {
            const int kk = k - 2 * HY * TXH;
            const int cc = kk % (2 * H);
            ly = HY + kk / (2 * H);
            lx = cc < H ? cc : TX + cc;
        }
        if (!hv[s]) lx = ly = 0;
        hL[s] = ly * TXH + lx;
        const int hx = wrapg(x0 - H + lx, nx);
        const int hy = L::DIM == 3 ? wrapg(y0 - HY + ly, ny) : 0;
        hX[s][0] = wrap1(hx - 1, nx); hX[s][1] = hx; hX[s][2] = wrap1(hx + 1, nx);
        if (L::DIM == 3) {
            hY[s][0] = wrap1(hy - 1, ny) * nx; hY[s][1] = hy * nx; hY[s][2] = wrap1(hy + 1, ny) * nx;
        } else {
            hY[s][0] = hY[s][1] = hY[s][2] = 0;
        }
    }

    // Pulled populations of the own site: fr[k] holds plane (collided + k)
    // for k = 0..H; fr[H + 1] receives the next plane, whose loads are in
    // flight while the current plane is collided (software pipelining: the
    // memory latency of plane p + H + 1 overlaps the arithmetic of plane p).
    R fr[H + 2][Q];
    R hr[NHT][Q];

    // issue the Q loads of the populations arriving at the site with offsets
    // (Xo, Yo) in the plane whose wrapped neighbour-plane offsets are P
    auto pull = [&](const int(&Xo)[3], const int(&Yo)[3], const int(&P)[3], R(&f)[Q]) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const unsigned e = unsigned(P[1 - op<L>(i)] + Yo[1 - oy<L>(i)] + Xo[1 - ox<L>(i)]);
            f[i] = R(buf_load(rs, e * ES, unsigned(i * stride) * ES, S()));
        }
    };
    // rho - sum_i s_i of pulled populations, in a fixed order: the moving
    // populations first, the rest population last.  In FP32 storage the rest
    // deviation carries the density contrast between the phases (|delta_0|
    // up to ~2, against ~1e-2 for the others), so adding it last leaves one
    // rounding at its scale instead of one per term (the velocity error
    // against the FP64 oracle drops about threefold, at no cost).
    auto dens = [&](const R(&f)[Q]) -> RD {
        R s = sum0<R>();
#pragma unroll
        for (int i = 1; i < Q; i++) s += f[i];
        return RD(s) + RD(f[0]);
    };

    auto plane_offsets = [&](int p, int(&P)[3]) {
        P[0] = wrap1(p - 1, np) * psz;
        P[1] = p * psz;
        P[2] = wrap1(p + 1, np) * psz;
    };

    auto rho_at = [&](int lp, int lx, int ly) -> RD & {
        return rho_s[(unsigned(lp) % NR) * PL + ly * TXH + lx];
    };

    // local plane lp is global plane p0 - H + lp: issue the loads of its own
    // site (into f) or of its halo sites; store their densities (pg: the
    // global plane index of lp, wrapped)
    auto load_own = [&](int pg, R(&f)[Q]) {
        int P[3];
        plane_offsets(pg, P);
        pull(X, Y, P, f);
    };
    auto load_halo = [&](int pg) {
        int P[3];
        plane_offsets(pg, P);
#pragma unroll
        for (int s = 0; s < NHT; s++)
            if (hv[s]) pull(hX[s], hY[s], P, hr[s]);
    };
    auto store_rho = [&](int lp, const R(&f)[Q]) {
        RD *ring = rho_s + (unsigned(lp) % NR) * PL;
        ring[(ty + HY) * TXH + tx + H] = dens(f);
#pragma unroll
        for (int s = 0; s < NHT; s++)
            if (hv[s]) ring[hL[s]] = dens(hr[s]);
    };

    // prologue: densities of planes p0-H .. p0+H (own populations of
    // p0 .. p0+H kept in fr[0..H])
    // (uniform across the workgroup, and marked so for the compiler)
    auto gplane = [&](int lp) { return __builtin_amdgcn_readfirstlane(wrapg(p0 - H + lp, np)); };
    for (int lp = 0; lp < H; lp++) {
        load_own(gplane(lp), fr[H + 1]);
        load_halo(gplane(lp));
        store_rho(lp, fr[H + 1]);
    }
#pragma unroll
    for (int s = 0; s <= H; s++) {
        load_own(gplane(H + s), fr[s]);
        load_halo(gplane(H + s));
        store_rho(H + s, fr[s]);
    }

    // Global indices (wrapped) of the plane collided and of the load front,
    // advanced by one plane per iteration (uniform values: a compare and
    // select, not a division).
    int pg_c = gplane(H), pg_f = gplane(2 * H + 1);
    auto advance = [&](int &pg) { pg = pg + 1 == np ? 0 : pg + 1; };

    // One plane.  The register ring is indexed at compile time: plane H + k
    // lives in fr[k mod (H + 2)], so the loop below is unrolled H + 2 times
    // and no registers move between planes (moves of in-flight load targets
    // would force waits at the loop head).
    auto iteration = [&](const int k, auto phase, auto always_more) {
        constexpr int RING = H + 2;
        constexpr int C0 = decltype(phase)::value % RING;            // plane lc
        constexpr int CN = (decltype(phase)::value + H + 1) % RING;  // plane lc + H + 1
        const int lc = H + k;  // local index of the plane collided now
        const bool more = decltype(always_more)::value || k + 1 < npl;
        if (more) {
            load_own(pg_f, fr[CN]);  // plane lc + H + 1, consumed after the collision
            load_halo(pg_f);
        }
        __syncthreads();  // densities up to plane lc + H are in LDS
        const int lx = tx + H, ly = ty + HY;
        const RD rho_dd = rho_at(lc, lx, ly);
        const R rho_dev = R(rho_dd);
        R j[3] = {sum0<R>(), sum0<R>(), L::DIM == 3 ? sum0<R>() : R(0)};
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (L::ex[i]) j[0] += R(L::ex[i]) * fr[C0][i];
            if (L::ey[i]) j[1] += R(L::ey[i]) * fr[C0][i];
            if (L::ez[i]) j[2] += R(L::ez[i]) * fr[C0][i];
        }
        // gradient (per weight class, Eq. (xderiv)) and Laplacian
        // (Eq. (laplace)) from the density ring
        R sa[3] = {sum0<R>(), sum0<R>(), sum0<R>()}, so[3] = {sum0<R>(), sum0<R>(), sum0<R>()};
        R lap = sum0<R>();
#pragma unroll
        for (int i = 1; i < Q; i++) {
            // (the stencil weights sum to zero: differences to the centre)
            const R r = R(rho_at(lc + op<L>(i), lx + ox<L>(i), ly + oy<L>(i)) - rho_dd);
            R *acc = nnz<L>(i) == 1 ? sa : so;
            if (L::ex[i]) acc[0] += R(L::ex[i]) * r;
            if (L::ey[i]) acc[1] += R(L::ey[i]) * r;
            if (L::ez[i]) acc[2] += R(L::ez[i]) * r;
            lap += coef_lap<L>(c, i) * r;
        }
        R d[3];
#pragma unroll
        for (int a = 0; a < 3; a++) d[a] = a < L::DIM ? c.A * sa[a] + c.B * so[a] : R(0);
        const R g[3] = {R(0), R(0), R(0)};
        const int p = pg_c;
        const unsigned site = unsigned(p * psz + Y[1] + X[1]);
        // collided populations (stored below)
        R out[Q];
        const EqSite<R> es =
            collide<L, false>(c, rho_dev, j, d, lap, g, fr[C0], [&](int i, R v) { out[i] = v; });
        if (own && J.observe) {
            J.obs_rho[site] = double(rho_dd) + c.shift_sum;
            J.obs_vel[site] = double(es.u[0]);
            J.obs_vel[J.obs_stride + site] = double(es.u[1]);
            J.obs_vel[2 * J.obs_stride + site] = double(L::DIM == 3 ? es.u[2] : R(0));
        }
        // Densities of the next plane: its ring slot (plane lc+H+1) is read by
        // no thread in this iteration (the ring holds the H + 3 planes
        // lc - 1 .. lc + H + 1), so no barrier is needed before this store;
        // the next iteration's barrier publishes it.
        if (more) store_rho(lc + H + 1, fr[CN]);
        // Global stores after the wait for the prefetched loads: memory
        // counters retire in order, so a wait on a load issued before these
        // stores would also wait for their write acknowledgements.
        if (own && J.write_pops) {
#pragma unroll
            for (int i = 0; i < Q; i++) buf_store(rd, site * ES, unsigned(i * stride) * ES, S(out[i]));
        }
        advance(pg_c);
        advance(pg_f);
    };

    // Full groups of H + 2 planes, every one of which prefetches: the loads
    // and the waits for them are unconditional here, so the compiler's wait
    // counting knows that the register ring is complete at the loop head (a
    // runtime prefetch condition made it wait for the fresh loads before the
    // collision).  The last group checks the condition at run time.
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    using P2 = std::integral_constant<int, 2>;
    int k = 0;
    for (; k + H + 2 < npl; k += H + 2) {
        iteration(k, P0{}, std::true_type{});
        iteration(k + 1, P1{}, std::true_type{});
        iteration(k + 2, P2{}, std::true_type{});
    }
    for (; k < npl; k += H + 2) {
        iteration(k, P0{}, std::false_type{});
        if (k + 1 < npl) iteration(k + 1, P1{}, std::false_type{});
        if (k + 2 < npl) iteration(k + 2, P2{}, std::false_type{});
    }
}

// The equilibrium march for FP32 storage, with the density front's own
// populations staged by direct-to-LDS loads (buffer_load ... lds) into two
// staging planes, as in the forcing march: plane lc + 3 is issued in the
// iteration that collides plane lc and taken into the register ring in the
// next one, after its collision and before its stores, so the staged loads
// have about two planes of work to arrive and hold no registers meanwhile.
// Memory operations are issued unconditionally (out-of-range offsets where a
// lane has nothing to do), so that the compiler counts the outstanding ones
// exactly and leaves the newest staged plane in flight.
template <class L, class S, class R, int TX, int TY>
__device__ __forceinline__ void eq_tile_dma(const Job<R> &J, const Coefs<R> &c)
{
    constexpr int Q = L::Q;
    constexpr int H = 1;
    constexpr int HY = L::DIM == 3 ? H : 0;
    constexpr int TXH = TX + 2 * H, TYH = TY + 2 * HY;
    constexpr int PL = TXH * TYH;
    constexpr int NR = 4;                       // density planes lc - 1 .. lc + 2
    constexpr int NT = TX * TY;
    constexpr int NHALO = 2 * HY * TXH + 2 * H * TY;
    constexpr int NHT = (NHALO + NT - 1) / NT;
    constexpr unsigned ES = sizeof(S);
    constexpr int RING = 2;                     // planes lc, lc + 1 (lc + 2 taken into lc's slot)
    constexpr int SPL = Q * NT;                 // floats per staging plane
    constexpr unsigned OOR = 0xFFFFFFFFu - (ES - 1);

    // FP32 arithmetic: densities in the ring as FP64 (the FP32 sum of the
    // moving deviations plus the rest one, not rounded at the scale of
    // rho - sum s_i), stencils on differences to the centre taken in FP64
    using RD = std::conditional_t<sizeof(R) == 4 && LBM_EQ_RING64, double, R>;
    __shared__ RD rho_s[NR * PL];
    __shared__ float stage0[SPL], stage1[SPL];

    const S *src = static_cast<const S *>(J.src);
    S *dst = static_cast<S *>(J.dst);
    const long long stride = J.stride;
    const int nx = J.nx, ny = J.ny, np = J.np;
    const int psz = nx * ny;
    const int x0 = J.x0, y0 = J.y0, p0 = J.p0, npl = J.npl;
    const __amdgpu_buffer_rsrc_t rs = pop_rsrc(src, J.bytes);
    const __amdgpu_buffer_rsrc_t rd = pop_rsrc(dst, J.bytes);

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int X[3], Y[3];
    const int gx = wrapg(x0 + tx, nx);
    const int gy = L::DIM == 3 ? wrapg(y0 + ty, ny) : 0;
    X[0] = wrap1(gx - 1, nx); X[1] = gx; X[2] = wrap1(gx + 1, nx);
    if (L::DIM == 3) {
        Y[0] = wrap1(gy - 1, ny) * nx; Y[1] = gy * nx; Y[2] = wrap1(gy + 1, ny) * nx;
    } else {
        Y[0] = Y[1] = Y[2] = 0;
    }
    const bool own = (x0 + tx < nx) && (L::DIM == 2 || y0 + ty < ny);

    int hX[NHT][3], hY[NHT][3], hL[NHT];
    bool hv[NHT];
#pragma unroll
    for (int s = 0; s < NHT; s++) {
        const int k = tid + s * NT;
        hv[s] = k < NHALO;
        int lx = 0, ly = 0;
        if (k < HY * TXH) {
            ly = k / TXH;
            lx = k % TXH;
        } else if (k < 2 * HY * TXH) {
            const int kk = k - HY * TXH;
            ly = TY + HY + kk / TXH;
            lx = kk % TXH;
        } else {
            const int kk = k - 2 * HY * TXH;
            const int cc = kk % (2 * H);
            ly = HY + kk / (2 * H);
            lx = cc < H ? cc : TX + cc;
        }
        if (!hv[s]) lx = ly = 0;
        hL[s] = ly * TXH + lx;
        const int hx = wrapg(x0 - H + lx, nx);
        const int hy = L::DIM == 3 ? wrapg(y0 - HY + ly, ny) : 0;
        hX[s][0] = wrap1(hx - 1, nx); hX[s][1] = hx; hX[s][2] = wrap1(hx + 1, nx);
        if (L::DIM == 3) {
            hY[s][0] = wrap1(hy - 1, ny) * nx; hY[s][1] = hy * nx; hY[s][2] = wrap1(hy + 1, ny) * nx;
        } else {
            hY[s][0] = hY[s][1] = hY[s][2] = 0;
        }
    }

    S fr[RING][Q];   // own populations: plane lc + k in fr[(phase + k) % RING]
    S dl[Q];         // own populations of the first plane (density only)
    S hr[NHT][Q];    // halo populations loaded for densities

    auto pull = [&](const int(&Xo)[3], const int(&Yo)[3], const int(&P)[3], S(&f)[Q], bool valid) {
        const unsigned oor = valid ? 0u : OOR;
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const unsigned e = unsigned(P[1 - op<L>(i)] + Yo[1 - oy<L>(i)] + Xo[1 - ox<L>(i)]);
            f[i] = buf_load(rs, (e * ES) | oor, unsigned(i * stride) * ES, S());
        }
    };
    auto dens = [&](const S(&f)[Q]) -> RD {
        R s = sum0<R>();
#pragma unroll
        for (int i = 1; i < Q; i++) s += R(f[i]);
        return RD(s) + RD(R(f[0]));
    };
    auto plane_offsets = [&](int p, int(&P)[3]) {
        P[0] = wrap1(p - 1, np) * psz;
        P[1] = p * psz;
        P[2] = wrap1(p + 1, np) * psz;
    };
    auto rho_at = [&](int lp, int lx, int ly) -> RD & {
        return rho_s[(unsigned(lp) % NR) * PL + ly * TXH + lx];
    };
    auto load_own = [&](int pg, S(&f)[Q]) {
        int P[3];
        plane_offsets(pg, P);
        pull(X, Y, P, f, true);
    };
    auto load_halo = [&](int pg, bool valid) {
        int P[3];
        plane_offsets(pg, P);
#pragma unroll
        for (int s = 0; s < NHT; s++) pull(hX[s], hY[s], P, hr[s], valid && hv[s]);
    };
    auto store_rho = [&](int lp, const S(&f)[Q]) {
        RD *ring = rho_s + (unsigned(lp) % NR) * PL;
        ring[(ty + HY) * TXH + tx + H] = dens(f);
#pragma unroll
        for (int s = 0; s < NHT; s++)
            if (hv[s]) ring[hL[s]] = dens(hr[s]);
    };
    auto dma_front = [&](int pg, auto buf, bool valid) {
        const unsigned oor = valid ? 0u : OOR;
        int P[3];
        plane_offsets(pg, P);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const unsigned e = unsigned(P[1 - op<L>(i)] + Y[1 - oy<L>(i)] + X[1 - ox<L>(i)]);
            float *const dst_l = (decltype(buf)::value ? stage1 : stage0) + i * NT + wave * 64;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)dst_l, 4,
                                                     (e * ES) | oor, unsigned(i * stride) * ES, 0, 0);
        }
    };
    auto take_front = [&](int lp, auto buf, S(&f)[Q]) {
#pragma unroll
        for (int i = 0; i < Q; i++) f[i] = decltype(buf)::value ? stage1[i * NT + tid] : stage0[i * NT + tid];
        store_rho(lp, f);
    };

    auto gplane = [&](int lp) { return __builtin_amdgcn_readfirstlane(wrapg(p0 - H + lp, np)); };
    // prologue: densities of local planes 0 .. 2H (global p0 - 1 .. p0 + 1;
    // the own populations of planes H, H + 1 stay in the ring), and the
    // staged plane 2H + 1, taken in the first iteration (from stage1)
    load_own(gplane(0), dl);
    load_halo(gplane(0), true);
    store_rho(0, dl);
    __builtin_amdgcn_sched_barrier(0);
    load_own(gplane(1), fr[0]);
    load_halo(gplane(1), true);
    store_rho(1, fr[0]);
    __builtin_amdgcn_sched_barrier(0);
    load_own(gplane(2), fr[1]);
    load_halo(gplane(2), true);
    store_rho(2, fr[1]);
    dma_front(gplane(3), std::true_type{}, npl > 1);

    // global planes of the collision, of the halo front taken this
    // iteration (lc + 2) and of the staged plane issued (lc + 3)
    int pg_c = gplane(H), pg_f = gplane(2 * H + 1), pg_f2 = gplane(2 * H + 2);
    auto advance = [&](int &pg) { pg = pg + 1 == np ? 0 : pg + 1; };

    auto iteration = [&](const int k, auto phase) {
        constexpr int C0 = decltype(phase)::value % RING;  // plane lc (lc + 2 after the take)
        using SbIssue = std::integral_constant<bool, decltype(phase)::value % 2 != 0>;
        using SbTake = std::integral_constant<bool, decltype(phase)::value % 2 == 0>;
        const int lc = H + k;
        const bool more = k + 1 < npl;
        // halo populations of plane lc + 2, consumed after the collision
        load_halo(pg_f, more);
        lds_sync();  // densities up to plane lc + 1 in LDS
        // own populations of plane lc + 3, taken in the next iteration
        dma_front(pg_f2, SbIssue{}, k + 2 < npl);
        const int lx = tx + H, ly = ty + HY;
        const RD rho_dd = rho_at(lc, lx, ly);
        const R rho_dev = R(rho_dd);
        S(&fc)[Q] = fr[C0];
        R j[3] = {sum0<R>(), sum0<R>(), L::DIM == 3 ? sum0<R>() : R(0)};
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (L::ex[i]) j[0] += R(L::ex[i]) * R(fc[i]);
            if (L::ey[i]) j[1] += R(L::ey[i]) * R(fc[i]);
            if (L::ez[i]) j[2] += R(L::ez[i]) * R(fc[i]);
        }
        R sa[3] = {sum0<R>(), sum0<R>(), sum0<R>()}, so[3] = {sum0<R>(), sum0<R>(), sum0<R>()};
        R lap = sum0<R>();
#pragma unroll
        for (int i = 1; i < Q; i++) {
            // (the stencil weights sum to zero: differences to the centre)
            const R r = R(rho_at(lc + op<L>(i), lx + ox<L>(i), ly + oy<L>(i)) - rho_dd);
            R *acc = nnz<L>(i) == 1 ? sa : so;
            if (L::ex[i]) acc[0] += R(L::ex[i]) * r;
            if (L::ey[i]) acc[1] += R(L::ey[i]) * r;
            if (L::ez[i]) acc[2] += R(L::ez[i]) * r;
            lap += coef_lap<L>(c, i) * r;
        }
        R d[3];
#pragma unroll
        for (int a = 0; a < 3; a++) d[a] = a < L::DIM ? c.A * sa[a] + c.B * so[a] : R(0);
        const R g[3] = {R(0), R(0), R(0)};
        const unsigned site = unsigned(pg_c * psz + Y[1] + X[1]);
        R fin[Q], out[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) fin[i] = R(fc[i]);
        const EqSite<R> es = collide<L, false>(c, rho_dev, j, d, lap, g, fin, [&](int i, R v) { out[i] = v; });
        if (own && J.observe) {
            J.obs_rho[site] = double(rho_dd) + c.shift_sum;
            J.obs_vel[site] = double(es.u[0]);
            J.obs_vel[J.obs_stride + site] = double(es.u[1]);
            J.obs_vel[2 * J.obs_stride + site] = double(L::DIM == 3 ? es.u[2] : R(0));
        }
        // plane lc + 2 into this plane's ring slot (its ring-of-densities slot
        // held plane lc - 2, read by no thread since the barrier above),
        // before the stores, so that waiting for its staged loads leaves
        // plane lc + 3's in flight
        if (more) take_front(lc + H + 1, SbTake{}, fc);
        const unsigned soor = (own && J.write_pops) ? 0u : OOR;
#pragma unroll
        for (int i = 0; i < Q; i++) buf_store(rd, (site * ES) | soor, unsigned(i * stride) * ES, S(out[i]));
        advance(pg_c);
        advance(pg_f);
        advance(pg_f2);
    };

    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    for (int k = 0; k < npl; k += RING) {
        iteration(k, P0{});
        if (k + 1 < npl) iteration(k + 1, P1{});
    }
}

} // namespace lbm

#include "lbm_force.h"

namespace lbm {

#ifndef LBM_EQ_DMA
#define LBM_EQ_DMA 1
#endif
// D2Q9 keeps the register march: its staging plane is a single row, the
// autotuned marches are short (4-16 rows per work item) and the staging's
// deeper prologue costs more than it hides (batched uneven D2Q9 FP32 drops:
// 0.366 against 0.397 ms per full-batch step).
#ifndef LBM_EQ_DMA_2D
#define LBM_EQ_DMA_2D 0
#endif

// The step of one tile: the forcing scheme's march (lbm_force.h) or the
// equilibrium scheme's (FP32 storage: with staged loads).
template <class L, int SCHEME, class S, class R, int TX, int TY>
__device__ __forceinline__ void tile_step(const Job<R> &J, const Coefs<R> &c)
{
    constexpr int NT = TX * TY, Q = L::Q, PLE = (TX + 2) * (TY + (L::DIM == 3 ? 2 : 0));
    constexpr int RDS = sizeof(R) == 4 && LBM_EQ_RING64 ? 8 : int(sizeof(R));  // ring element
    constexpr bool EQ_DMA =
        LBM_EQ_DMA && (L::DIM == 3 || LBM_EQ_DMA_2D) && sizeof(S) == 4 &&
        (2 * Q * NT * 4 + 4 * PLE * RDS) <= 160 * 1024;
    if constexpr (SCHEME == SCHEME_FORCE)
        force_tile<L, S, R, TX, TY>(J, c);
    else if constexpr (EQ_DMA)
        eq_tile_dma<L, S, R, TX, TY>(J, c);
    else
        eq_tile<L, S, R, TX, TY>(J, c);
}

// One problem: workgroup b takes tile (b mod tiles_x, ...) of chunk b / tiles.
template <class L, int SCHEME, class S, class R, int TX, int TY>
__global__ __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(step_waves_per_eu<L, SCHEME, S, R>())))
void step_kernel(StepArgs<R> A)
{
    // XCD-aware order: consecutive workgroup ids go to different XCDs, so
    // give each XCD a contiguous run of tiles (neighbours share halos in L2).
    const int nb = A.tiles_x * A.tiles_y * A.chunks;
    int b = blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int tile_x = b % A.tiles_x;
    const int tile_y = (b / A.tiles_x) % A.tiles_y;
    const int chunk = b / (A.tiles_x * A.tiles_y);
    Job<R> J;
    J.src = A.src;
    J.dst = A.dst;
    J.stride = A.n;
    J.bytes = unsigned((long long)L::Q * A.n * (long long)sizeof(S));
    J.obs_rho = A.obs_rho;
    J.obs_vel = A.obs_vel;
    J.obs_stride = A.n;
    J.nx = A.nx;
    J.ny = A.ny;
    J.np = A.np;
    J.x0 = tile_x * TX;
    J.y0 = tile_y * TY;
    J.p0 = chunk * A.cp;
    J.npl = min(A.cp, A.np - J.p0);
    J.write_pops = A.write_pops;
    J.observe = A.observe;
    if (J.npl <= 0) return;
    tile_step<L, SCHEME, S, R, TX, TY>(J, A.c);
}

// ---- many independent problems in one persistent launch --------------------

struct BatchProblem {
    long long off;       // first site of the problem in the concatenated arrays
    int nx, ny, np;      // kernel geometry (D2Q9: ny = 1, np = lattice ny)
    int tiles_x, tiles_y, chunks, cp;
    int item0;           // first work item of the problem
};

template <class R> struct BatchArgs {
    const void *src;
    void *dst;
    long long stride;             // total sites (elements between directions)
    double *obs_rho, *obs_vel;    // concatenated observation fields
    const BatchProblem *prob;     // [nprob]
    const Coefs<R> *coefs;        // [nprob]
    const int *active;            // [nprob]; 0 = skip (converged or stopped)
    int nprob, nitems;
    int write_pops, observe;
};

// Persistent grid: workgroup g takes work items g, g + G, ...; an item is
// one tile x chunk of one problem (binary search over item0).  Items of
// inactive problems are skipped, so converged problems keep their state.
template <class L, int SCHEME, class S, class R, int TX, int TY>
__global__ __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<L, SCHEME, S>())))
void batch_step_kernel(BatchArgs<R> B)
{
    for (int w = blockIdx.x; w < B.nitems; w += gridDim.x) {
        int lo = 0, hi = B.nprob - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (B.prob[mid].item0 <= w) lo = mid; else hi = mid - 1;
        }
        const int k = lo;
        if (!B.active[k]) continue;
        const BatchProblem P = B.prob[k];
        const int item = w - P.item0;
        const int tile_x = item % P.tiles_x;
        const int tile_y = (item / P.tiles_x) % P.tiles_y;
        const int chunk = item / (P.tiles_x * P.tiles_y);
        Job<R> J;
        J.src = static_cast<const S *>(B.src) + P.off;
        J.dst = static_cast<S *>(B.dst) + P.off;
        J.stride = B.stride;
        J.bytes = unsigned(((long long)L::Q * B.stride - P.off) * (long long)sizeof(S));
        J.obs_rho = B.obs_rho ? B.obs_rho + P.off : nullptr;
        J.obs_vel = B.obs_vel ? B.obs_vel + P.off : nullptr;
        J.obs_stride = B.stride;
        J.nx = P.nx;
        J.ny = P.ny;
        J.np = P.np;
        J.x0 = tile_x * TX;
        J.y0 = tile_y * TY;
        J.p0 = chunk * P.cp;
        J.npl = min(P.cp, P.np - J.p0);
        J.write_pops = B.write_pops;
        J.observe = B.observe;
        tile_step<L, SCHEME, S, R, TX, TY>(J, B.coefs[k]);
        __syncthreads();  // the LDS rings are reused by the next item
    }
}

} // namespace lbm

// The D3Q19 instances of step_kernel (every launch shape and arithmetic):
// instantiated in lbm_step3d.hip, a translation unit of their own that the
// build compiles with another machine-scheduler strategy, and declared
// extern where they are launched.
#define LBM_STEP3D_SHAPES(X, SCH, S, R) \
    X(SCH, S, R, 64, 4) X(SCH, S, R, 32, 8) X(SCH, S, R, 64, 8) X(SCH, S, R, 32, 16) X(SCH, S, R, 128, 4)
#define LBM_STEP3D_INSTANCES(X)                                                                   \
    LBM_STEP3D_SHAPES(X, 0, double, double) LBM_STEP3D_SHAPES(X, 0, float, float)                \
    LBM_STEP3D_SHAPES(X, 0, float, double) LBM_STEP3D_SHAPES(X, 1, double, double)               \
    LBM_STEP3D_SHAPES(X, 1, float, float) LBM_STEP3D_SHAPES(X, 1, float, double)
