// lbm_force.h -- the fused step of the momentum-conserving forcing scheme
// (section "Using a forcing method"), marching plane by plane.
//
// Included by lbm_step.h (uses its Job, buffer and wrap helpers).
//
// The body force g_a = -sum_b d_b (M_ab - delta_ab M_cc / 2), M_ab = kappa
// d_a rho d_b rho, needs the density two sites away, so a workgroup keeps
// the densities of its tile plus a 2-site halo in an LDS ring of planes.
// The tensor T_ab = M_ab - delta_ab M_cc / 2 is formed once per plane on the
// tile plus a 1-site border (one LDS plane); every site then adds that
// plane's share of the force stencil to the forces of the three planes that
// see it: r + e_i lies in plane q for r in plane q - e_iz.  A site's force
// is complete once the plane above it has been added, so only three force
// partial sums (9 registers) and the own gradient travel with the march,
// and each T value read from LDS serves up to three directions.
//
// Own populations: the density front runs three planes ahead of the
// collision, so each thread keeps its site's populations of four planes in
// a register ring (the newest in flight during the collision).
//
// Measured on D3Q19 256^3 (64 x 8 tiles, 128 planes per workgroup), against
// a march that kept the gradient and T of three planes in LDS (88 KB) and
// summed the force per direction: FP32 0.593 against 0.638 ms per step, FP64
// 1.330 against 1.518 ms.  Loading each plane twice instead (for its
// density, and again from L2 for its collision, 57 registers of loads
// instead of 76) ran at 0.744 ms: the second reads left L2.
#pragma once

namespace lbm {

#ifndef LBM_FORCE_DMA
#define LBM_FORCE_DMA 1
#endif
// FP32 arithmetic with an FP64 density ring (see the ring below)
#ifndef LBM_FORCE_RING64
#define LBM_FORCE_RING64 1
#endif
// D2Q9 keeps the register march (short marches, see lbm_step.h): 1024^2 FP32
// forcing 0.0196 against 0.0243 ms per step.
#ifndef LBM_FORCE_DMA_2D
#define LBM_FORCE_DMA_2D 0
#endif

template <class L, class S, class R, int TX, int TY>
__device__ __forceinline__ void force_tile(const Job<R> &J, const Coefs<R> &c)
{
    constexpr int Q = L::Q, DIM = L::DIM;
    constexpr int H = 2;                           // density halo
    constexpr int HY = DIM == 3 ? H : 0;           // in-plane y halo
    constexpr int TXH = TX + 2 * H, TYH = TY + 2 * HY;
    constexpr int PL = TXH * TYH;                  // LDS sites per density plane
    constexpr int NR = 5;                          // density planes lc - 1 .. lc + 3
    constexpr int GY = DIM == 3 ? 1 : 0;           // T plane in-plane y border
    constexpr int TXG = TX + 2, TYG = TY + 2 * GY;
    constexpr int GPL = TXG * TYG;                 // LDS sites per T plane
    constexpr int NTC = DIM == 3 ? 6 : 2;          // independent T components
    constexpr int NT = TX * TY;
    constexpr int NHALO = 2 * HY * TXH + 2 * H * TY;
    constexpr int NHT = (NHALO + NT - 1) / NT;     // density-halo sites per thread
    constexpr int NBORD = GPL - NT;                // T-plane sites outside the tile
    constexpr int NBT = (NBORD + NT - 1) / NT;
    constexpr unsigned ES = sizeof(S);
    constexpr int RING = H + 2;                    // own-population planes in registers
    // FP32: the density front's populations travel by direct-to-LDS loads
    // into two staging planes, so plane lc + 4 is in flight while plane
    // lc + 3 is taken into registers (see below); needs every halo site in
    // one pass of the threads and the staging to fit the LDS.
    constexpr int SPL = Q * NT;                    // floats per staging plane
    // FP32 arithmetic: the density ring holds FP64 values (the rest
    // deviation added to the FP32 sum of the moving ones without rounding),
    // and the stencils take differences to the centre in FP64 before
    // rounding them: an FP32 ring would round every density at its own
    // scale (|rho - sum s_i| up to ~3, 1.2e-7) and the Laplacian and
    // gradients would carry those roundings into the equilibrium and the
    // force every step
    using RD = std::conditional_t<sizeof(R) == 4 && LBM_FORCE_RING64, double, R>;
    constexpr bool DMA = LBM_FORCE_DMA && (DIM == 3 || LBM_FORCE_DMA_2D) && sizeof(S) == 4 &&
                         2 * SPL * 4 + NR * PL * sizeof(RD) + NTC * GPL * sizeof(R) <= 160 * 1024;

    __shared__ RD rho_s[NR * PL];
    // T components: 3D xx, yy, zz, xy, xz, yz; 2D xx, xy (T_yy = -T_xx)
    __shared__ R t_s[NTC * GPL];
    __shared__ float stage0[DMA ? SPL : 1], stage1[DMA ? SPL : 1];

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
    int X[3], Y[3];
    const int gx = wrapg(x0 + tx, nx);
    const int gy = DIM == 3 ? wrapg(y0 + ty, ny) : 0;
    X[0] = wrap1(gx - 1, nx); X[1] = gx; X[2] = wrap1(gx + 1, nx);
    if (DIM == 3) {
        Y[0] = wrap1(gy - 1, ny) * nx; Y[1] = gy * nx; Y[2] = wrap1(gy + 1, ny) * nx;
    } else {
        Y[0] = Y[1] = Y[2] = 0;
    }
    const bool own = (x0 + tx < nx) && (DIM == 2 || y0 + ty < ny);

    // density-halo sites of this thread (fixed for the march)
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
        const int hy = DIM == 3 ? wrapg(y0 - HY + ly, ny) : 0;
        hX[s][0] = wrap1(hx - 1, nx); hX[s][1] = hx; hX[s][2] = wrap1(hx + 1, nx);
        if (DIM == 3) {
            hY[s][0] = wrap1(hy - 1, ny) * nx; hY[s][1] = hy * nx; hY[s][2] = wrap1(hy + 1, ny) * nx;
        } else {
            hY[s][0] = hY[s][1] = hY[s][2] = 0;
        }
    }
    // T-plane border sites of this thread: the rows above and below the tile
    // (3D), then the columns left and right of it
    int bL[NBT];
    bool bv[NBT];
#pragma unroll
    for (int s = 0; s < NBT; s++) {
        const int k = tid + s * NT;
        bv[s] = k < NBORD;
        int lx = 0, ly = 0;
        if (DIM == 3 && k < 2 * TXG) {
            ly = k < TXG ? 0 : TYG - 1;
            lx = k % TXG;
        } else {
            const int kk = DIM == 3 ? k - 2 * TXG : k;
            ly = GY + kk / 2;
            lx = (kk % 2) ? TXG - 1 : 0;
        }
        bL[s] = bv[s] ? ly * TXG + lx : 0;
    }

    // Populations are held as stored (S) and widened where used, so FP32
    // storage with FP64 arithmetic keeps its register ring in FP32.
    S fr[RING][Q];   // own populations: plane lc + k in fr[(phase + k) % RING]
    S dl[Q];         // own populations of the first planes (densities only)
    S hr[NHT][Q];    // halo populations loaded for densities

    // Byte offset past every buffer: loads from it return zero and stores to
    // it are dropped by the buffer range check.  The DMA march issues its
    // memory operations unconditionally, with this offset where a lane has
    // nothing to load or store, so that every wave issues the same sequence
    // and the compiler can count outstanding operations exactly (a
    // conditional one makes it wait for all of them, prefetch included).
    constexpr unsigned OOR = 0xFFFFFFFFu - (ES - 1);
    // (offsets are or-ed with OOR rather than selected, which the compiler
    // would turn into branches around duplicated loads)
    auto pull = [&](const int(&Xo)[3], const int(&Yo)[3], const int(&P)[3], S(&f)[Q], bool valid = true) {
        const unsigned oor = valid ? 0u : OOR;
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const unsigned e = unsigned(P[1 - op<L>(i)] + Yo[1 - oy<L>(i)] + Xo[1 - ox<L>(i)]);
            f[i] = buf_load(rs, (e * ES) | oor, unsigned(i * stride) * ES, S());
        }
    };
    // rho - sum_i s_i: moving populations first, the rest population last
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
    auto load_own = [&](int pg, S(&f)[Q]) {
        int P[3];
        plane_offsets(pg, P);
        pull(X, Y, P, f);
    };
    auto load_halo = [&](int pg, bool valid = true) {
        int P[3];
        plane_offsets(pg, P);
#pragma unroll
        for (int s = 0; s < NHT; s++) {
            if constexpr (DMA)
                pull(hX[s], hY[s], P, hr[s], valid && hv[s]);
            else if (hv[s])
                pull(hX[s], hY[s], P, hr[s]);
        }
    };
    auto rho_at = [&](int lp, int lx, int ly) -> RD & {
        return rho_s[(unsigned(lp) % NR) * PL + ly * TXH + lx];
    };
    auto store_rho = [&](int lp, const S(&f)[Q]) {
        RD *ring = rho_s + (unsigned(lp) % NR) * PL;
        ring[(ty + HY) * TXH + tx + H] = dens(f);
#pragma unroll
        for (int s = 0; s < NHT; s++)
            if (hv[s]) ring[hL[s]] = dens(hr[s]);
    };

    // Direct-to-LDS loads of a plane's own and halo populations into staging
    // plane sb: wave w's lane l writes direction i of site w * 64 + l (own)
    // or of halo site w * 64 + l, so each thread later reads back what its
    // own wave wrote.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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
    // take a staged plane's own populations into f and their density into
    // the ring, with the halo densities from the halo loads in hr
    auto take_front = [&](int lp, auto buf, S(&f)[Q]) {
#pragma unroll
        for (int i = 0; i < Q; i++) f[i] = decltype(buf)::value ? stage1[i * NT + tid] : stage0[i * NT + tid];
        store_rho(lp, f);
    };

    // gradient of the density plane lp at density-ring site (rx, ry), summed
    // per weight class (Eq. (xderiv); 3D: the A, B stencil)
    auto gradient = [&](int lp, int rx, int ry, R(&d)[3]) {
        R sa[3] = {sum0<R>(), sum0<R>(), sum0<R>()}, so[3] = {sum0<R>(), sum0<R>(), sum0<R>()};
        // the stencil's weights sum to zero, so the centre may be subtracted
        const RD rc = rho_at(lp, rx, ry);
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const R r = R(rho_at(lp + op<L>(i), rx + ox<L>(i), ry + oy<L>(i)) - rc);
            R *acc = nnz<L>(i) == 1 ? sa : so;
            if (L::ex[i]) acc[0] += R(L::ex[i]) * r;
            if (L::ey[i]) acc[1] += R(L::ey[i]) * r;
            if (L::ez[i]) acc[2] += R(L::ez[i]) * r;
        }
#pragma unroll
        for (int a = 0; a < 3; a++) d[a] = a < DIM ? c.A * sa[a] + c.B * so[a] : R(0);
    };
    // T at T-plane site k from the gradient d
    auto store_t = [&](int k, const R(&d)[3]) {
        if constexpr (DIM == 3) {
            const R h = R(0.5) * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            t_s[0 * GPL + k] = c.kappa * (d[0] * d[0] - h);
            t_s[1 * GPL + k] = c.kappa * (d[1] * d[1] - h);
            t_s[2 * GPL + k] = c.kappa * (d[2] * d[2] - h);
            t_s[3 * GPL + k] = c.kappa * (d[0] * d[1]);
            t_s[4 * GPL + k] = c.kappa * (d[0] * d[2]);
            t_s[5 * GPL + k] = c.kappa * (d[1] * d[2]);
        } else {
            t_s[0 * GPL + k] = c.kappa * (R(0.5) * (d[0] * d[0] - d[1] * d[1]));
            t_s[1 * GPL + k] = c.kappa * (d[0] * d[1]);
        }
    };
    // T of local plane lp on the tile and its border; returns the own
    // site's gradient (d_own) and Laplacian (lap_own, Eqs. (laplace),
    // (laplacian3d)), which share the neighbour densities
    auto fill_t = [&](int lp, R(&d_own)[3], R &lap_own) {
        {
            const int rx = tx + H, ry = ty + HY;
            const RD rc = rho_at(lp, rx, ry);
            R sa[3] = {sum0<R>(), sum0<R>(), sum0<R>()}, so[3] = {sum0<R>(), sum0<R>(), sum0<R>()};
            R la = sum0<R>();
#pragma unroll
            for (int i = 1; i < Q; i++) {
                const R r = R(rho_at(lp + op<L>(i), rx + ox<L>(i), ry + oy<L>(i)) - rc);
                R *acc = nnz<L>(i) == 1 ? sa : so;
                if (L::ex[i]) acc[0] += R(L::ex[i]) * r;
                if (L::ey[i]) acc[1] += R(L::ey[i]) * r;
                if (L::ez[i]) acc[2] += R(L::ez[i]) * r;
                la += coef_lap<L>(c, i) * r;
            }
#pragma unroll
            for (int a = 0; a < 3; a++) d_own[a] = a < DIM ? c.A * sa[a] + c.B * so[a] : R(0);
            lap_own = la;
        }
        store_t((ty + GY) * TXG + tx + 1, d_own);
#pragma unroll
        for (int s = 0; s < NBT; s++) {
            if (!bv[s]) continue;
            const int lx = bL[s] % TXG, ly = bL[s] / TXG;
            R d[3];
            gradient(lp, lx + (H - 1), ly + (HY - GY), d);
            store_t(bL[s], d);
        }
    };
    // component (a, b) of T at T-plane site k
    auto t_at = [&](int a, int b, int k) -> R {
        if constexpr (DIM == 3) {
            const int comp = a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
            return t_s[comp * GPL + k];
        } else {
            const R v = t_s[(a == b ? 0 : 1) * GPL + k];
            return (a == 1 && b == 1) ? -v : v;
        }
    };
    // Add the T plane q's share of sum_i c_i sum_b e_ib T_ab(r + e_i) to the
    // force sums of the own site in planes q - 1 (gm), q (g0) and q + 1 (gp).
    auto add_t = [&](R(&gm)[3], R(&g0)[3], R(&gp)[3]) {
        const int k0 = (ty + GY) * TXG + tx + 1;
#pragma unroll
        for (int pos = 0; pos < 9; pos++) {
            const int px = pos % 3 - 1, py = pos / 3 - 1;
            if (DIM == 2 && py != 0) continue;
            const int k = k0 + py * TXG + px;
#pragma unroll
            for (int i = 1; i < Q; i++) {
                if (ox<L>(i) != px || oy<L>(i) != py) continue;
                const R cf = coef_force<L>(c, i);
                R *acc = op<L>(i) > 0 ? gm : (op<L>(i) < 0 ? gp : g0);
#pragma unroll
                for (int a = 0; a < DIM; a++) {
                    R t = sum0<R>();
#pragma unroll
                    for (int b = 0; b < DIM; b++)
                        if (ecomp<L>(i, b)) t += R(ecomp<L>(i, b)) * t_at(a, b, k);
                    acc[a] += cf * t;
                }
            }
            // one in-plane position at a time: the scheduler would otherwise
            // hoist all of the plane's LDS reads and hold them in registers
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    auto gplane = [&](int lp) { return __builtin_amdgcn_readfirstlane(wrapg(p0 - H + lp, np)); };

    // Prologue: densities of local planes 0 .. 2H (global p0 - 2 .. p0 + 2;
    // the own populations of planes H .. 2H stay in the ring), then T of
    // planes H - 1 and H, which also give the gradient and Laplacian of
    // plane H.
    R gc[3], g1[3], g2[3], dc[3], dn[3], lapc, lapn;
#pragma unroll
    for (int a = 0; a < 3; a++) gc[a] = g1[a] = g2[a] = sum0<R>();
#pragma unroll
    for (int lp = 0; lp <= 2 * H; lp++) {
        S(&f)[Q] = lp >= H ? fr[(lp - H) % RING] : dl;
        load_own(gplane(lp), f);
        load_halo(gplane(lp));
        store_rho(lp, f);
        __builtin_amdgcn_sched_barrier(0);
    }
    // DMA: plane 2H + 1, taken in the first iteration (whose staging plane
    // to take is stage1, see the iteration)
    if constexpr (DMA) dma_front(gplane(2 * H + 1), std::true_type{}, npl > 1);
    lds_sync();
    {
        R dd[3], ld, gx0[3] = {sum0<R>(), sum0<R>(), sum0<R>()};
        fill_t(H - 1, dd, ld);
        lds_sync();
        add_t(gx0, gx0, gc);  // plane H - 1 reaches plane H through e_iz = -1
        lds_sync();
        fill_t(H, dc, lapc);
        lds_sync();
        add_t(gx0, gc, g1);
    }

    // global planes of the collision and of the density front (lc + H + 1;
    // DMA: lc + H + 2 is the one issued)
    int pg_c = gplane(H), pg_f = gplane(2 * H + 1), pg_f2 = gplane(2 * H + 2);
    auto advance = [&](int &pg) { pg = pg + 1 == np ? 0 : pg + 1; };

    auto iteration = [&](const int k, auto phase) {
        constexpr int C0 = decltype(phase)::value % RING;             // plane lc
        constexpr int CN = (decltype(phase)::value + H + 1) % RING;  // plane lc + H + 1
        const int lc = H + k;
        const bool more = k + 1 < npl;
        S(&fc)[Q] = fr[C0];
        S(&fn)[Q] = fr[CN];
        // lc = H + phase (mod RING), RING even: the staging plane of plane
        // lc + 4 (issued here) and of plane lc + 3 (taken here)
        using SbIssue = std::integral_constant<bool, decltype(phase)::value % 2 != 0>;
        using SbTake = std::integral_constant<bool, decltype(phase)::value % 2 == 0>;
        // Density front: plane lc + 3, in flight during this plane's work
        // (software pipelining: its memory latency overlaps the collision).
        // DMA: only its halo populations here; the own ones were staged.
        if constexpr (DMA)
            load_halo(pg_f, more);
        else if (more) {
            load_own(pg_f, fn);
            load_halo(pg_f);
        }
        lds_sync();  // densities up to plane lc + 2 in LDS; T plane free
        // DMA: own populations of plane lc + 4 into the staging plane taken
        // in the previous iteration (every thread is past its reads), taken
        // in the next iteration: in flight for two planes of work
        if constexpr (DMA) dma_front(pg_f2, SbIssue{}, k + 2 < npl);
        fill_t(lc + 1, dn, lapn);
        lds_sync();  // T of plane lc + 1 in LDS
        add_t(gc, g1, g2);
        // DMA: plane lc + 3 into the ring now, before this plane's stores,
        // so that waiting for its staged loads leaves plane lc + 4's in flight
        // (memory counters retire in order)
        if (DMA && more) take_front(lc + H + 1, SbTake{}, fn);

        const RD rho_dd = rho_at(lc, tx + H, ty + HY);
        const R rho_dev = R(rho_dd);
        R j[3] = {sum0<R>(), sum0<R>(), DIM == 3 ? sum0<R>() : R(0)};
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (L::ex[i]) j[0] += R(L::ex[i]) * R(fc[i]);
            if (L::ey[i]) j[1] += R(L::ey[i]) * R(fc[i]);
            if (L::ez[i]) j[2] += R(L::ez[i]) * R(fc[i]);
        }
        R g[3];
#pragma unroll
        for (int a = 0; a < 3; a++) g[a] = a < DIM ? -gc[a] : R(0);

        const unsigned site = unsigned(pg_c * psz + Y[1] + X[1]);
        const bool st = own && J.write_pops;
        const unsigned soor = st ? 0u : OOR;
        R fin[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) fin[i] = R(fc[i]);
        const EqSite<R> es = collide<L, true>(c, rho_dev, j, dc, lapc, g, fin, [&](int i, R v) {
            if constexpr (DMA)
                buf_store(rd, (site * ES) | soor, unsigned(i * stride) * ES, S(v));
            else if (st)
                buf_store(rd, site * ES, unsigned(i * stride) * ES, S(v));
        });
        if (own && J.observe) {
            J.obs_rho[site] = double(rho_dd) + c.shift_sum;
            const R h = R(0.5) / es.rho;
            J.obs_vel[site] = double(es.u[0] + h * g[0]);
            J.obs_vel[J.obs_stride + site] = double(es.u[1] + h * g[1]);
            J.obs_vel[2 * J.obs_stride + site] = double(DIM == 3 ? es.u[2] + h * g[2] : R(0));
        }
        // Densities of plane lc + 3: its ring slot held plane lc - 2, which no
        // thread reads in this iteration; the next iteration's first barrier
        // publishes them.  The population stores above went out after the
        // front's loads, so waiting for those loads does not wait for them.
        if (!DMA && more) store_rho(lc + H + 1, fn);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            gc[a] = g1[a];
            g1[a] = g2[a];
            g2[a] = sum0<R>();
            dc[a] = dn[a];
        }
        lapc = lapn;
        advance(pg_c);
        advance(pg_f);
        advance(pg_f2);
    };

    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    using P2 = std::integral_constant<int, 2>;
    using P3 = std::integral_constant<int, 3>;
    // the register ring is indexed at compile time: unrolled by its length
    // (splitting off full groups with unconditional prefetches, as the
    // equilibrium march does, made this kernel spill)
    for (int k = 0; k < npl; k += RING) {
        iteration(k, P0{});
        if (k + 1 < npl) iteration(k + 1, P1{});
        if (k + 2 < npl) iteration(k + 2, P2{});
        if (k + 3 < npl) iteration(k + 3, P3{});
    }
}

} // namespace lbm
