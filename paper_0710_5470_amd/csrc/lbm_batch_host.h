// lbm_batch_host.h -- host side of the batched runner (included once, at the
// end of lbm_capi.hip, so it shares that file's helpers).
//
// Many independent problems (same lattice, scheme, storage and arithmetic;
// their own extent and a, b, T, kappa, tau) live in concatenated SoA arrays.
// One persistent launch per step walks a flat list of (problem, tile, plane
// chunk) work items.  A check every K steps (K even) measures each problem's
// residual and retires converged, diverging or non-finite problems on the
// device; the K steps plus the check are captured once in a hipGraph and
// replayed, with one 4-byte readback (the number of active problems) per
// replay.

#include <vector>

#include "lbm_batch.h"

struct lbm_batch {
    int nprob;
    lbm_params base;               // shared lattice / scheme / storage / compute
    std::vector<lbm_params> pp;
    hipStream_t stream;
    char *ws;
    long long ntot;
    std::vector<long long> off, nsite;
    std::vector<int> gnx, gny, gnp; // kernel geometry per problem
    int tile, cp, nitems, grid;
    int cus;                       // compute units of the device the batch runs on
    size_t o_a, o_b, o_rho, o_vel, o_prev, o_prob, o_coef, o_act, o_all, o_state, o_off, o_ns,
        o_b_coef, o_stats, o_count, total;
    hipGraphExec_t exec;
    int graph_K;
    bool graph_ok;
    int cur;
    long long steps;
    bool all_active;  // false once lbm_batch_run has retired a problem
};

namespace {

size_t batch_layout(lbm_batch *bt)
{
    const int q = bt->base.lattice;
    const size_t es = bt->base.storage == LBM_STORE_F64 ? 8 : 4;
    const size_t nt = (size_t)bt->ntot, np = (size_t)bt->nprob;
    size_t o = 0;
    bt->o_a = o; o += align_up(nt * q * es);
    bt->o_b = o; o += align_up(nt * q * es);
    bt->o_rho = o; o += align_up(nt * 8);
    bt->o_vel = o; o += align_up(3 * nt * 8);
    bt->o_prev = o; o += align_up(3 * nt * 8);
    bt->o_prob = o; o += align_up(np * sizeof(BatchProblem));
    bt->o_coef = o; o += align_up(np * sizeof(Coefs<double>));
    bt->o_act = o; o += align_up(np * sizeof(int));
    bt->o_all = o; o += align_up(np * sizeof(int));
    bt->o_state = o; o += align_up(np * sizeof(BatchState));
    bt->o_off = o; o += align_up(np * 8);
    bt->o_ns = o; o += align_up(np * 8);
    bt->o_b_coef = o; o += align_up(np * 8);
    bt->o_stats = o; o += align_up(np * 4 * 8);
    bt->o_count = o; o += align_up(64);
    bt->total = o;
    return o;
}

template <class T> T *bptr(lbm_batch *bt, size_t o) { return reinterpret_cast<T *>(bt->ws + o); }

bool batch_compatible(const lbm_params *a, const lbm_params *b)
{
    return a->lattice == b->lattice && a->scheme == b->scheme && a->storage == b->storage &&
           a->compute == b->compute;
}

void batch_geometry(lbm_batch *bt)
{
    bt->gnx.resize(bt->nprob);
    bt->gny.resize(bt->nprob);
    bt->gnp.resize(bt->nprob);
    for (int k = 0; k < bt->nprob; k++) {
        const lbm_params &p = bt->pp[k];
        bt->gnx[k] = p.nx;
        bt->gny[k] = p.lattice == LBM_D2Q9 ? 1 : p.ny;
        bt->gnp[k] = p.lattice == LBM_D2Q9 ? p.ny : p.nz;
    }
}

// Work-item table for the current tile / planes choice.
int batch_items(lbm_batch *bt)
{
    TileShape t = tile_shape(bt->base.lattice, bt->tile);
    std::vector<BatchProblem> h(bt->nprob);
    int items = 0;
    for (int k = 0; k < bt->nprob; k++) {
        BatchProblem P{};
        P.off = bt->off[k];
        P.nx = bt->gnx[k];
        P.ny = bt->gny[k];
        P.np = bt->gnp[k];
        // at most cp planes per chunk, the problem's planes spread evenly
        // over its chunks (no short last chunk paying a full prologue)
        P.chunks = (P.np + std::min(bt->cp, P.np) - 1) / std::min(bt->cp, P.np);
        P.cp = (P.np + P.chunks - 1) / P.chunks;
        P.tiles_x = (P.nx + t.tx - 1) / t.tx;
        P.tiles_y = (P.ny + t.ty - 1) / t.ty;
        P.item0 = items;
        items += P.tiles_x * P.tiles_y * P.chunks;
        h[k] = P;
    }
    bt->nitems = items;
    if (hipMemcpyAsync(bptr<BatchProblem>(bt, bt->o_prob), h.data(), h.size() * sizeof(BatchProblem),
                       hipMemcpyHostToDevice, bt->stream) != hipSuccess)
        return LBM_E_DEVICE;
    if (hipStreamSynchronize(bt->stream) != hipSuccess) return LBM_E_DEVICE;
    bt->graph_ok = false;
    return LBM_OK;
}

// Planes per work item while `active` problems remain.  A step's latency is
// one work item's plane march, so when few problems are left the march is
// shortened (halving from cp0, not below LBM_TAIL_MIN_PLANES) until there
// are again LBM_TAIL_ITEMS_PER_CU work items per compute unit (512 drops of
// 128^2 from 26 planes per item: 2.26 s to residual 1e-10 with 2 items per
// CU, 2.21 s with 4, 2.15 s with 8).  Results do not depend on the launch.
#ifndef LBM_TAIL_ITEMS_PER_CU
#define LBM_TAIL_ITEMS_PER_CU 8
#endif
#ifndef LBM_TAIL_MIN_PLANES
#define LBM_TAIL_MIN_PLANES 4
#endif

int tail_planes(const lbm_batch *bt, int active, int cp0)
{
    const TileShape t = tile_shape(bt->base.lattice, bt->tile);
    double tiles = 0.0, planes = 0.0;
    for (int k = 0; k < bt->nprob; k++) {
        tiles += double((bt->gnx[k] + t.tx - 1) / t.tx) * ((bt->gny[k] + t.ty - 1) / t.ty);
        planes += bt->gnp[k];
    }
    tiles /= bt->nprob;
    planes /= bt->nprob;
    const double target = double(LBM_TAIL_ITEMS_PER_CU) * std::max(1, bt->cus);
    int cp = cp0;
    while (cp > LBM_TAIL_MIN_PLANES && active * tiles * std::ceil(planes / cp) < target)
        cp = std::max(cp / 2, LBM_TAIL_MIN_PLANES);
    return cp;
}

template <class L, int SCH, class S, class R, int TX, int TY>
void batch_launch_one(lbm_batch *bt, const BatchArgs<R> &a)
{
    auto kern = batch_step_kernel<L, SCH, S, R, TX, TY>;
    // resident workgroups per CU of this instantiation (same on every gfx950)
    static const int per_cu = [&] {
        int v = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kern, TX * TY, 0) == hipSuccess
                   ? std::max(1, v)
                   : 1;
    }();
    int g = per_cu * std::max(1, bt->cus);
    g = std::min(g, std::max(1, a.nitems));
    bt->grid = g;
    kern<<<g, TX * TY, 0, bt->stream>>>(a);
}

template <class L, int SCH, class S, class R> void batch_launch_tiles(lbm_batch *bt, const BatchArgs<R> &a)
{
    if constexpr (L::DIM == 2) {
        switch (bt->tile) {
        case 0: batch_launch_one<L, SCH, S, R, 64, 1>(bt, a); break;
        case 1: batch_launch_one<L, SCH, S, R, 128, 1>(bt, a); break;
        default: batch_launch_one<L, SCH, S, R, 256, 1>(bt, a); break;
        }
    } else {
        switch (bt->tile) {
        case 0: batch_launch_one<L, SCH, S, R, 64, 4>(bt, a); break;
        case 1: batch_launch_one<L, SCH, S, R, 32, 8>(bt, a); break;
        case 2: batch_launch_one<L, SCH, S, R, 64, 8>(bt, a); break;
        case 3: batch_launch_one<L, SCH, S, R, 32, 16>(bt, a); break;
        default: batch_launch_one<L, SCH, S, R, 128, 4>(bt, a); break;
        }
    }
}

template <class L, int SCH, class S, class R>
void batch_step_t(lbm_batch *bt, const void *src, void *dst, int write, int observe, double *orho,
                  double *ovel, const int *active)
{
    BatchArgs<R> a{};
    a.src = src;
    a.dst = dst;
    a.stride = bt->ntot;
    a.obs_rho = orho;
    a.obs_vel = ovel;
    a.prob = bptr<BatchProblem>(bt, bt->o_prob);
    a.coefs = bptr<Coefs<R>>(bt, bt->o_coef);
    a.active = active;
    a.nprob = bt->nprob;
    a.nitems = bt->nitems;
    a.write_pops = write;
    a.observe = observe;
    batch_launch_tiles<L, SCH, S, R>(bt, a);
}

template <class L, int SCH>
void batch_step_l(lbm_batch *bt, int write, int observe, double *orho, double *ovel, const int *active)
{
    void *cur = bt->ws + (bt->cur ? bt->o_b : bt->o_a);
    void *nxt = bt->ws + (bt->cur ? bt->o_a : bt->o_b);
    if (bt->base.storage == LBM_STORE_F64)
        batch_step_t<L, SCH, double, double>(bt, cur, nxt, write, observe, orho, ovel, active);
    else if (bt->base.compute == LBM_COMPUTE_F64)
        batch_step_t<L, SCH, float, double>(bt, cur, nxt, write, observe, orho, ovel, active);
    else
        batch_step_t<L, SCH, float, float>(bt, cur, nxt, write, observe, orho, ovel, active);
}

// one batched step of every active problem (write) and / or an observation
void batch_step(lbm_batch *bt, int write, int observe, double *orho, double *ovel, const int *active)
{
    bool d3 = bt->base.lattice == LBM_D3Q19, fo = bt->base.scheme == LBM_SCHEME_FORCE;
    if (!d3 && !fo) batch_step_l<D2Q9, SCHEME_EQ>(bt, write, observe, orho, ovel, active);
    if (!d3 && fo) batch_step_l<D2Q9, SCHEME_FORCE>(bt, write, observe, orho, ovel, active);
    if (d3 && !fo) batch_step_l<D3Q19, SCHEME_EQ>(bt, write, observe, orho, ovel, active);
    if (d3 && fo) batch_step_l<D3Q19, SCHEME_FORCE>(bt, write, observe, orho, ovel, active);
    if (write) bt->cur ^= 1;
}

template <class L, class S> void batch_init_one(lbm_batch *bt, int k, const Coefs<double> &cd,
                                                const double *rho0, const double *u0)
{
    Geom g{bt->gnx[k], bt->gny[k], bt->gnp[k], bt->nsite[k], bt->ntot};
    S *dst = reinterpret_cast<S *>(bt->ws + bt->o_a) + bt->off[k];
    const double *u = u0 ? u0 + bt->off[k] : nullptr;
    if (bt->base.scheme == LBM_SCHEME_EQ)
        init_kernel<L, SCHEME_EQ, S><<<grid1(g.n), 256, 0, bt->stream>>>(g, cd, rho0 + bt->off[k], u, dst);
    else
        init_kernel<L, SCHEME_FORCE, S><<<grid1(g.n), 256, 0, bt->stream>>>(g, cd, rho0 + bt->off[k], u, dst);
}

int batch_capture(lbm_batch *bt, int K, double tol, int patience, long long grace, long long max_steps)
{
    if (bt->graph_ok) {
        bt->graph_ok = false;
        if (hipGraphExecDestroy(bt->exec) != hipSuccess) return LBM_E_DEVICE;
    }
    hipGraph_t graph;
    if (hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return LBM_E_DEVICE;
    int *count = bptr<int>(bt, bt->o_count);
    const int *act = bptr<int>(bt, bt->o_act);
    double *rho = bptr<double>(bt, bt->o_rho), *vel = bptr<double>(bt, bt->o_vel),
           *prev = bptr<double>(bt, bt->o_prev);
    batch_zero_kernel<<<1, 64, 0, bt->stream>>>(count);
    for (int s = 0; s < K - 1; s++) batch_step(bt, 1, 0, nullptr, nullptr, act);
    batch_step(bt, 1, 1, rho, prev, act);  // observe t, advance to t + 1
    batch_step(bt, 0, 1, rho, vel, act);   // observe t + 1
    batch_check_kernel<<<bt->nprob, RED_THREADS, 0, bt->stream>>>(
        bptr<long long>(bt, bt->o_off), bptr<long long>(bt, bt->o_ns), bptr<double>(bt, bt->o_b_coef),
        bt->ntot, rho, vel, prev, bptr<BatchState>(bt, bt->o_state), K, tol, patience, grace,
        max_steps, count);
    batch_flags_kernel<<<(bt->nprob + 255) / 256, 256, 0, bt->stream>>>(
        bptr<BatchState>(bt, bt->o_state), bptr<int>(bt, bt->o_act), bt->nprob);
    hipError_t e = hipStreamEndCapture(bt->stream, &graph);
    if (e != hipSuccess) return LBM_E_DEVICE;
    e = hipGraphInstantiate(&bt->exec, graph, nullptr, nullptr, 0);
    const hipError_t ed = hipGraphDestroy(graph);
    if (e != hipSuccess || ed != hipSuccess) return LBM_E_DEVICE;
    bt->graph_ok = true;
    bt->graph_K = K;
    return LBM_OK;
}

} // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(int nprob, const lbm_params *pp)
{
    if (nprob < 1 || !pp) return 0;
    lbm_batch tmp{};
    tmp.nprob = nprob;
    tmp.base = pp[0];
    tmp.ntot = 0;
    for (int k = 0; k < nprob; k++) {
        if (!valid_params(&pp[k]) || !batch_compatible(&pp[0], &pp[k])) return 0;
        tmp.ntot += (long long)pp[k].nx * pp[k].ny * pp[k].nz;
    }
    double es = pp[0].storage == LBM_STORE_F64 ? 8.0 : 4.0;
    if ((double)tmp.ntot * es * pp[0].lattice >= 4294967296.0) return 0;
    return batch_layout(&tmp);
}

int lbm_batch_init(lbm_batch **out, int nprob, const lbm_params *pp, void *dev_workspace,
                   size_t bytes, void *stream, const double *dev_rho0, const double *dev_u0)
{
    if (!out || nprob < 1 || !pp || !dev_workspace || !dev_rho0 || !stream) return LBM_E_INVAL;
    *out = nullptr;
    size_t need = lbm_batch_workspace_bytes(nprob, pp);
    if (need == 0) return LBM_E_INVAL;
    if (bytes < need) return LBM_E_NOMEM;
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN) return LBM_E_INVAL;
    lbm_batch *bt = new (std::nothrow) lbm_batch();
    if (!bt) return LBM_E_NOMEM;
    bt->nprob = nprob;
    bt->all_active = true;
    bt->base = pp[0];
    bt->pp.assign(pp, pp + nprob);
    bt->stream = static_cast<hipStream_t>(stream);
    bt->ws = static_cast<char *>(dev_workspace);
    bt->off.resize(nprob);
    bt->nsite.resize(nprob);
    bt->ntot = 0;
    for (int k = 0; k < nprob; k++) {
        bt->off[k] = bt->ntot;
        bt->nsite[k] = (long long)pp[k].nx * pp[k].ny * pp[k].nz;
        bt->ntot += bt->nsite[k];
    }
    batch_layout(bt);
    batch_geometry(bt);
    bt->graph_ok = false;
    bt->cur = 0;
    bt->steps = 0;
    {
        int dev = 0;
        bt->cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&bt->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            delete bt;
            return LBM_E_DEVICE;
        }
    }
    bt->tile = pp[0].tile >= 0 ? pp[0].tile : 0;
    bt->cp = pp[0].planes_per_block > 0 ? pp[0].planes_per_block : 16;
    std::vector<double> bcoef(nprob);
    for (int k = 0; k < nprob; k++) bcoef[k] = pp[k].b;
    auto fail = [&](int rc) {
        delete bt;
        return rc;
    };
    if (hipMemcpyAsync(bptr<long long>(bt, bt->o_off), bt->off.data(), nprob * 8, hipMemcpyHostToDevice,
                       bt->stream) != hipSuccess ||
        hipMemcpyAsync(bptr<long long>(bt, bt->o_ns), bt->nsite.data(), nprob * 8,
                       hipMemcpyHostToDevice, bt->stream) != hipSuccess ||
        hipMemcpyAsync(bptr<double>(bt, bt->o_b_coef), bcoef.data(), nprob * 8, hipMemcpyHostToDevice,
                       bt->stream) != hipSuccess)
        return fail(LBM_E_DEVICE);
    // validate every initial density segment and take its mean
    batch_field_stats_kernel<<<nprob, RED_THREADS, 0, bt->stream>>>(
        bptr<long long>(bt, bt->o_off), bptr<long long>(bt, bt->o_ns), bptr<double>(bt, bt->o_b_coef),
        dev_rho0, bptr<double>(bt, bt->o_stats));
    std::vector<double> stats(4 * nprob);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(stats.data(), bptr<double>(bt, bt->o_stats), stats.size() * 8,
                       hipMemcpyDeviceToHost, bt->stream) != hipSuccess ||
        hipStreamSynchronize(bt->stream) != hipSuccess)
        return fail(LBM_E_DEVICE);
    std::vector<Coefs<double>> cd(nprob);
    std::vector<Coefs<float>> cf(nprob);
    for (int k = 0; k < nprob; k++) {
        if (stats[4 * k + 3] != 0.0) return fail(LBM_E_INVAL);
        double mean = stats[4 * k] / double(bt->nsite[k]);
        double rs = std::isnan(pp[k].rho_shift) ? mean : pp[k].rho_shift;
        cd[k] = make_coefs(&pp[k]);
        make_shift(&pp[k], cd[k], rs);
        cf[k] = to_float(cd[k], pp[k].lattice);
    }
    const bool f32math = bt->base.storage != LBM_STORE_F64 && bt->base.compute == LBM_COMPUTE_NATIVE;
    hipError_t e = f32math ? hipMemcpyAsync(bptr<char>(bt, bt->o_coef), cf.data(), nprob * sizeof(Coefs<float>),
                                            hipMemcpyHostToDevice, bt->stream)
                           : hipMemcpyAsync(bptr<char>(bt, bt->o_coef), cd.data(), nprob * sizeof(Coefs<double>),
                                            hipMemcpyHostToDevice, bt->stream);
    if (e != hipSuccess) return fail(LBM_E_DEVICE);
    std::vector<BatchState> st(nprob);
    std::vector<int> ones(nprob, 1);
    for (int k = 0; k < nprob; k++) {
        st[k] = BatchState{};
        st[k].active = 1;
    }
    if (hipMemcpyAsync(bptr<BatchState>(bt, bt->o_state), st.data(), nprob * sizeof(BatchState),
                       hipMemcpyHostToDevice, bt->stream) != hipSuccess ||
        hipMemcpyAsync(bptr<int>(bt, bt->o_act), ones.data(), nprob * 4, hipMemcpyHostToDevice,
                       bt->stream) != hipSuccess ||
        hipMemcpyAsync(bptr<int>(bt, bt->o_all), ones.data(), nprob * 4, hipMemcpyHostToDevice,
                       bt->stream) != hipSuccess)
        return fail(LBM_E_DEVICE);
    bool d3 = bt->base.lattice == LBM_D3Q19, f64 = bt->base.storage == LBM_STORE_F64;
    for (int k = 0; k < nprob; k++) {
        if (!d3 && f64) batch_init_one<D2Q9, double>(bt, k, cd[k], dev_rho0, dev_u0);
        if (!d3 && !f64) batch_init_one<D2Q9, float>(bt, k, cd[k], dev_rho0, dev_u0);
        if (d3 && f64) batch_init_one<D3Q19, double>(bt, k, cd[k], dev_rho0, dev_u0);
        if (d3 && !f64) batch_init_one<D3Q19, float>(bt, k, cd[k], dev_rho0, dev_u0);
    }
    if (hipGetLastError() != hipSuccess) return fail(LBM_E_DEVICE);
    int rc = batch_items(bt);
    if (rc != LBM_OK) return fail(rc);
    *out = bt;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *bt, long long nsteps)
{
    if (!bt || nsteps < 0) return LBM_E_INVAL;
    // A retired problem is skipped, so its state stays in the buffer it was
    // in; an odd count would leave the active problems in the other one.
    if ((nsteps & 1) && !bt->all_active) return LBM_E_STATE;
    for (long long s = 0; s < nsteps; s++) batch_step(bt, 1, 0, nullptr, nullptr, bptr<int>(bt, bt->o_act));
    bt->steps += nsteps;
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_batch_run(lbm_batch *bt, double tol, int check_every, long long max_steps, int patience,
                  long long grace, long long *host_steps, double *host_residual, int *host_status)
{
    if (!bt || !(tol >= 0.0) || check_every < 1 || max_steps < 1) return LBM_E_INVAL;
    int K = check_every + (check_every & 1);  // even: a replay returns to the same buffer
    int rc = batch_capture(bt, K, tol, patience, grace, max_steps);
    if (rc != LBM_OK) return rc;
    int *count = bptr<int>(bt, bt->o_count);
    int h_count = bt->nprob;
    long long done = 0;
    const int cp0 = bt->cp;
    while (h_count > 0 && done < max_steps) {
        const int cp = tail_planes(bt, h_count, cp0);
        if (cp != bt->cp) {
            bt->cp = cp;
            if ((rc = batch_items(bt)) != LBM_OK ||
                (rc = batch_capture(bt, K, tol, patience, grace, max_steps)) != LBM_OK)
                return rc;
        }
        if (hipGraphLaunch(bt->exec, bt->stream) != hipSuccess) return LBM_E_DEVICE;
        done += K;
        if (hipMemcpyAsync(&h_count, count, sizeof(int), hipMemcpyDeviceToHost, bt->stream) != hipSuccess ||
            hipStreamSynchronize(bt->stream) != hipSuccess)
            return LBM_E_DEVICE;
    }
    bt->steps += done;
    bt->all_active = h_count == bt->nprob;
    if (bt->cp != cp0) {  // the caller's launch again for later calls
        bt->cp = cp0;
        if ((rc = batch_items(bt)) != LBM_OK) return rc;
    }
    std::vector<BatchState> st(bt->nprob);
    if (hipMemcpyAsync(st.data(), bptr<BatchState>(bt, bt->o_state), st.size() * sizeof(BatchState),
                       hipMemcpyDeviceToHost, bt->stream) != hipSuccess ||
        hipStreamSynchronize(bt->stream) != hipSuccess)
        return LBM_E_DEVICE;
    for (int k = 0; k < bt->nprob; k++) {
        if (host_steps) host_steps[k] = st[k].steps;
        if (host_residual) host_residual[k] = st[k].residual;
        if (host_status) host_status[k] = st[k].status;
    }
    return LBM_OK;
}

int lbm_batch_reactivate(lbm_batch *bt)
{
    if (!bt) return LBM_E_INVAL;
    std::vector<BatchState> st(bt->nprob);
    std::vector<int> ones(bt->nprob, 1);
    for (auto &s : st) {
        s = BatchState{};
        s.active = 1;
    }
    if (hipMemcpyAsync(bptr<BatchState>(bt, bt->o_state), st.data(), st.size() * sizeof(BatchState),
                       hipMemcpyHostToDevice, bt->stream) != hipSuccess ||
        hipMemcpyAsync(bptr<int>(bt, bt->o_act), ones.data(), ones.size() * 4, hipMemcpyHostToDevice,
                       bt->stream) != hipSuccess ||
        hipStreamSynchronize(bt->stream) != hipSuccess)
        return LBM_E_DEVICE;
    bt->all_active = true;
    return LBM_OK;
}

int lbm_batch_moments(lbm_batch *bt, double *dev_rho, double *dev_vel)
{
    if (!bt || !dev_rho || !dev_vel) return LBM_E_INVAL;
    batch_step(bt, 0, 1, dev_rho, dev_vel, bptr<int>(bt, bt->o_all));
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

int lbm_batch_max_spurious_u(lbm_batch *bt, double *host_out)
{
    if (!bt || !host_out) return LBM_E_INVAL;
    double *vel = bptr<double>(bt, bt->o_vel), *stats = bptr<double>(bt, bt->o_stats);
    batch_step(bt, 0, 1, bptr<double>(bt, bt->o_rho), vel, bptr<int>(bt, bt->o_all));
    batch_maxvel_kernel<<<bt->nprob, RED_THREADS, 0, bt->stream>>>(
        bptr<long long>(bt, bt->o_off), bptr<long long>(bt, bt->o_ns), bt->ntot, vel, stats);
    std::vector<double> h(2 * (size_t)bt->nprob);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h.data(), stats, h.size() * sizeof(double), hipMemcpyDeviceToHost, bt->stream) !=
            hipSuccess ||
        hipStreamSynchronize(bt->stream) != hipSuccess)
        return LBM_E_DEVICE;
    bool bad = false;
    for (int k = 0; k < bt->nprob; k++) {
        host_out[k] = h[2 * k];
        bad = bad || h[2 * k + 1] != 0.0;
    }
    return bad ? LBM_E_NONFINITE : LBM_OK;
}

long long lbm_batch_offset(const lbm_batch *bt, int k)
{
    if (!bt || k < 0 || k > bt->nprob) return -1;
    return k == bt->nprob ? bt->ntot : bt->off[k];
}

int lbm_batch_set_launch(lbm_batch *bt, int tile, int planes)
{
    if (!bt || tile >= lbm_tile_count(bt->base.lattice)) return LBM_E_INVAL;
    if (tile >= 0) bt->tile = tile;
    if (planes > 0) bt->cp = planes;
    return batch_items(bt);
}

int lbm_batch_get_launch(const lbm_batch *bt, int *tile, int *planes, int *items)
{
    if (!bt) return LBM_E_INVAL;
    if (tile) *tile = bt->tile;
    if (planes) *planes = bt->cp;
    if (items) *items = bt->nitems;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch *bt)
{
    if (!bt) return LBM_E_INVAL;
    const hipError_t e = bt->graph_ok ? hipGraphExecDestroy(bt->exec) : hipSuccess;
    delete bt;
    return e == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

} // extern "C"
