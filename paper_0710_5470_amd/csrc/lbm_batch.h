// lbm_batch.h -- device kernels of the batched runner: per-problem field
// statistics, the convergence check that retires problems, and a counter
// reset that graph capture can record (no memset nodes in captured graphs).
#pragma once

#include "lbm_aux.h"

namespace lbm {

enum BatchStatus { BST_RUNNING = 0, BST_CONVERGED = 1, BST_MAXSTEPS = 2, BST_DIVERGED = 3, BST_NONFINITE = 4 };

struct BatchState {
    int active;        // 1 while the problem still steps
    int status;        // BatchStatus
    int rises;         // consecutive checks with a risen residual
    int pad;
    long long steps;   // steps taken while active
    double residual;   // last max |vel(t+1) - vel(t)|
    double max_vel;    // last max |vel|
    double best;       // smallest residual seen after the grace period (0: none yet)
};

// A residual counts as risen when it exceeds the smallest one seen so far by
// this factor: a decaying oscillation (sound waves crossing the box) makes
// consecutive samples go up and down, a growing or stuck-high state does not
// come back down.
constexpr double RISE_FACTOR = 10.0;

// One workgroup per problem: sum, min, max and bad-site count of a field
// segment (initial density validation and the FP32 shift density).
__global__ __launch_bounds__(RED_THREADS) void batch_field_stats_kernel(const long long *off,
                                                                        const long long *nsite,
                                                                        const double *b_coef,
                                                                        const double *__restrict__ f,
                                                                        double *__restrict__ out)
{
    const int k = blockIdx.x;
    const long long o = off[k], n = nsite[k];
    const double b = b_coef[k];
    double v[4] = {0.0, INFINITY, -INFINITY, 0.0};
    const int ops[4] = {RED_SUM, RED_MIN, RED_MAX, RED_SUM};
    for (long long s = threadIdx.x; s < n; s += RED_THREADS) {
        double r = f[o + s];
        v[0] += r;
        v[1] = fmin(v[1], r);
        v[2] = fmax(v[2], r);
        v[3] += (!isfinite(r) || r <= 0.0 || b * r >= 1.0) ? 1.0 : 0.0;
    }
    block_reduce<4>(v, ops);
    if (threadIdx.x == 0)
        for (int j = 0; j < 4; j++) out[4 * k + j] = v[j];
}

// One workgroup per problem: max |vel| over the problem's sites and the
// number of non-finite velocity entries (written to out[2k], out[2k + 1]).
__global__ __launch_bounds__(RED_THREADS) void batch_maxvel_kernel(const long long *off,
                                                                   const long long *nsite, long long stride,
                                                                   const double *__restrict__ vel,
                                                                   double *__restrict__ out)
{
    const int k = blockIdx.x;
    const long long o = off[k], n = nsite[k];
    double v[2] = {0.0, 0.0};
    const int ops[2] = {RED_MAX, RED_SUM};
    for (long long s = threadIdx.x; s < n; s += RED_THREADS) {
        const long long q = o + s;
        const double a0 = vel[q], a1 = vel[stride + q], a2 = vel[2 * stride + q];
        const double sp = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        v[0] = isfinite(sp) ? fmax(v[0], sp) : INFINITY;
        v[1] += isfinite(sp) ? 0.0 : 1.0;
    }
    block_reduce<2>(v, ops);
    if (threadIdx.x == 0) {
        out[2 * k] = v[0];
        out[2 * k + 1] = v[1];
    }
}

__global__ void batch_zero_kernel(int *counter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// One workgroup per problem.  For active problems: residual
// max_r |vel(r,t+1) - vel(r,t)| and max |vel| over the problem's sites (FP64),
// then retire the problem when converged (residual <= tol), non-finite,
// rising for `patience` consecutive checks (after `grace` steps), or out of
// steps.  Active problems add themselves to *n_active.
__global__ __launch_bounds__(RED_THREADS) void batch_check_kernel(
    const long long *off, const long long *nsite, const double *b_coef, long long stride,
    const double *__restrict__ rho, const double *__restrict__ vel, const double *__restrict__ prev,
    BatchState *st, int steps_per_check, double tol, int patience, long long grace,
    long long max_steps, int *n_active)
{
    const int k = blockIdx.x;
    if (!st[k].active) return;
    const long long o = off[k], n = nsite[k];
    const double b = b_coef[k];
    double v[3] = {0.0, 0.0, 0.0};
    const int ops[3] = {RED_MAX, RED_MAX, RED_SUM};
    for (long long s = threadIdx.x; s < n; s += RED_THREADS) {
        const long long q = o + s;
        double r = rho[q];
        double a0 = vel[q], a1 = vel[stride + q], a2 = vel[2 * stride + q];
        double d0 = a0 - prev[q], d1 = a1 - prev[stride + q], d2 = a2 - prev[2 * stride + q];
        double sp = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        double dr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        v[0] = fmax(v[0], sp);
        v[1] = fmax(v[1], dr);
        v[2] += (!(isfinite(r) && isfinite(sp) && isfinite(dr)) || r <= 0.0 || b * r >= 1.0) ? 1.0 : 0.0;
    }
    block_reduce<3>(v, ops);
    if (threadIdx.x == 0) {
        BatchState s = st[k];
        s.steps += steps_per_check;
        s.max_vel = v[0];
        s.residual = v[1];
        if (v[2] != 0.0) {
            s.status = BST_NONFINITE;
        } else if (v[1] <= tol) {
            s.status = BST_CONVERGED;
        } else {
            const bool past_grace = s.steps > grace;
            s.rises = (past_grace && s.best > 0.0 && v[1] > RISE_FACTOR * s.best) ? s.rises + 1 : 0;
            if (past_grace && (s.best == 0.0 || v[1] < s.best)) s.best = v[1];
            if (patience > 0 && s.rises >= patience) s.status = BST_DIVERGED;
            else if (s.steps >= max_steps) s.status = BST_MAXSTEPS;
        }
        if (s.status != BST_RUNNING) s.active = 0;
        st[k] = s;
        if (s.active) atomicAdd(n_active, 1);
    }
}

// active flags for the step kernel (a plain int array)
__global__ void batch_flags_kernel(const BatchState *st, int *active, int nprob)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nprob) active[k] = st[k].active;
}

} // namespace lbm
