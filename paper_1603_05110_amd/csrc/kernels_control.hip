// Device-side control of one time step.  The decisions of the fixed point
// (Section 2.2: stop when the increment is small), of the Schwarz iteration
// (Section 5: stop when ||g^{k+1} - g^k|| < tol) and of the preconditioned
// update (eq. algo_pd) are taken by one-block kernels that write a StepCtl in
// device memory; every kernel of an iteration reads the flags first and
// returns at once when its phase is already complete.  The host can then
// enqueue a whole Schwarz iteration and synchronise once per iteration.
#include "osm_internal.h"

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ double block_sum(double v, double *red) {
    v = wsum(v);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

__global__ void step_init_kernel(StepCtl *c, StepCfg cfg) {
    if (threadIdx.x != 0) return;
    c->cfg = cfg;
    c->q_conv = 0; c->q_iter = 0; c->q_total = 0; c->q_fail = 0;
    c->r_done = 0; c->k = 0; c->k_done = 0; c->bad = 0; c->commit = 0;
    c->gm_total = 0;
    c->tq = cfg.tol_q;
    c->inc = 0.0; c->ref = 0.0; c->prev_rel = 1.0;
}

// Start of Schwarz iteration k: new fixed point, tolerance from the previous
// increment (inexact inner solves, option eta_q), GMRES cycle idle.
__global__ void iter_reset_kernel(StepCtl *c, GmresCtl *g) {
    if (threadIdx.x != 0) return;
    if (c->k_done || c->bad) return;
    c->q_conv = 0;
    c->q_iter = 0;
    c->q_fail = 0;
    c->r_done = 0;
    c->commit = 0;
    double t = c->cfg.tol_q;
    if (c->cfg.eta_q > 0.0) t = fmax(t, c->cfg.eta_q * fmin(1.0, c->prev_rel));
    c->tq = t;
    if (g) { g->done = 1; g->finished = 0; g->conv = 0; g->j = 0; g->total = 0; }
}

__global__ void copy_u_guarded_kernel(Phys P, const StripMeta *strips, const int *line_strip,
                                      const double2 *u, double2 *zeta, const StepCtl *c) {
    if (c->k_done || c->bad) return;
    int L = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= P.ny) return;
    StripMeta s = strips[line_strip[L]];
    int gl = s.line0 + (L - s.off);
    zeta[(long)L * P.ny + a] = u[(long)gl * P.ny + a];
}

// Fixed-point test of every strip from the per-line partial sums:
// converged when ||dzeta_j|| <= tq ||zeta_j|| for all strips j (or after
// fixed_q iterations).  One block.
__global__ void q_check_kernel(Phys P, const StripMeta *strips, const double *part, StepCtl *c) {
    if (c->q_conv || c->k_done || c->bad) return;
    __shared__ int notconv, nonfinite;
    if (threadIdx.x == 0) { notconv = 0; nonfinite = 0; }
    __syncthreads();
    double tq = c->tq;
    for (int j = threadIdx.x; j < P.nsub; j += blockDim.x) {
        StripMeta s = strips[j];
        double d = 0, z = 0, b = 0;
        for (int i = 0; i < s.nx; ++i) {
            d += part[3 * (s.off + i)];
            z += part[3 * (s.off + i) + 1];
            b += part[3 * (s.off + i) + 2];
        }
        if (b > 0 || !isfinite(d) || !isfinite(z)) atomicOr(&nonfinite, 1);
        if (!(sqrt(d) <= tq * sqrt(z))) atomicOr(&notconv, 1);
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    c->q_iter += 1;
    c->q_total += 1;
    if (nonfinite) { c->bad = 1; return; }
    bool conv = c->cfg.fixed_q > 0 ? (c->q_iter >= c->cfg.fixed_q) : !notconv;
    if (conv) c->q_conv = 1;
    else if (c->q_iter >= c->cfg.max_q) c->q_fail = 1;
}

// End of the Schwarz map: ||g^{k+1} - g^k||, ||g^{k+1}|| from the flux
// partials.  Classical algorithm: decide convergence and commit g <- R(g).
__global__ void flux_finalize_kernel(const double *part, int nt, StepCtl *c) {
    if (!c->q_conv || c->r_done || c->k_done || c->bad) return;
    __shared__ double red[16];
    double a = 0, b = 0;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) { a += part[2 * t]; b += part[2 * t + 1]; }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x != 0) return;
    c->r_done = 1;
    if (!c->cfg.classical) return;
    double inc = sqrt(a), ref = sqrt(b);
    if (!isfinite(inc)) { c->bad = 1; return; }
    c->commit = 1;
    c->k += 1;
    c->inc = inc;
    c->ref = ref;
    c->prev_rel = inc / fmax(ref, 1e-300);
    double thr = c->cfg.tol_k_rel ? c->cfg.tol_k * fmax(ref, 1e-300) : c->cfg.tol_k;
    if (c->cfg.fixed_k > 0) { if (c->k >= c->cfg.fixed_k) c->k_done = 1; }
    else if (inc < thr) c->k_done = 1;
}

__global__ void commit_kernel(long n, double2 *g, const double2 *gn, const StepCtl *c) {
    if (!c->commit) return;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) g[e] = gn[e];
}

// y = g - R(g) for the preconditioned update, and x = 0 / GMRES cycle reset.
__global__ void precond_rhs_kernel(long n, const double2 *g, const double2 *gn, double2 *y,
                                   double2 *x, const StepCtl *c) {
    if (c->r_done != 1 || c->k_done || c->bad) return;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) {
        double2 a = g[e], b = gn[e];
        y[e] = cd(a.x - b.x, a.y - b.y);
        x[e] = cd(0.0, 0.0);
    }
}

// g <- g - x after GMRES, with per-block partials of |x|^2, |g|^2.
__global__ void precond_update_kernel(long n, double2 *g, const double2 *x, double *part,
                                      const StepCtl *c, const GmresCtl *gc) {
    if (c->r_done != 1 || c->k_done || c->bad || !gc->finished || !gc->conv) return;
    __shared__ double red[16];
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double sx = 0, sg = 0;
    if (e < n) {
        double2 xv = x[e], gv = g[e];
        gv = cd(gv.x - xv.x, gv.y - xv.y);
        g[e] = gv;
        sx = xv.x * xv.x + xv.y * xv.y;
        sg = gv.x * gv.x + gv.y * gv.y;
    }
    sx = block_sum(sx, red);
    sg = block_sum(sg, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sx;
        part[2 * blockIdx.x + 1] = sg;
    }
}

__global__ void precond_finalize_kernel(const double *part, int nb, StepCtl *c,
                                        const GmresCtl *gc) {
    if (c->r_done != 1 || c->k_done || c->bad || !gc->finished || !gc->conv) return;
    __shared__ double red[16];
    double a = 0, b = 0;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) { a += part[2 * t]; b += part[2 * t + 1]; }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x != 0) return;
    double inc = sqrt(a), ref = sqrt(b);
    c->r_done = 2;
    c->gm_total += gc->total;
    if (!isfinite(inc)) { c->bad = 1; return; }
    c->k += 1;
    c->inc = inc;
    c->ref = ref;
    c->prev_rel = inc / fmax(ref, 1e-300);
    double thr = c->cfg.tol_k_rel ? c->cfg.tol_k * fmax(ref, 1e-300) : c->cfg.tol_k;
    if (c->cfg.fixed_k > 0) { if (c->k >= c->cfg.fixed_k) c->k_done = 1; }
    else if (inc < thr) c->k_done = 1;
}

}  // namespace

static inline dim3 vgrid(long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_step_init(hipStream_t st, StepCtl *c, const StepCfg &cfg) {
    hipLaunchKernelGGL(step_init_kernel, dim3(1), dim3(64), 0, st, c, cfg);
    return hipGetLastError();
}

hipError_t launch_iter_reset(hipStream_t st, StepCtl *c, GmresCtl *g) {
    hipLaunchKernelGGL(iter_reset_kernel, dim3(1), dim3(64), 0, st, c, g);
    return hipGetLastError();
}

hipError_t launch_copy_u_guarded(hipStream_t st, const Phys &P, const StripMeta *strips,
                                 const int *line_strip, const double2 *u, double2 *zeta,
                                 const StepCtl *c) {
    hipLaunchKernelGGL(copy_u_guarded_kernel, dim3((P.ny + 255) / 256, P.lt), dim3(256), 0, st,
                       P, strips, line_strip, u, zeta, c);
    return hipGetLastError();
}

hipError_t launch_q_check(hipStream_t st, const Phys &P, const StripMeta *strips,
                          const double *part, StepCtl *c) {
    hipLaunchKernelGGL(q_check_kernel, dim3(1), dim3(256), 0, st, P, strips, part, c);
    return hipGetLastError();
}

hipError_t launch_flux_finalize(hipStream_t st, const double *part, int nt, StepCtl *c) {
    hipLaunchKernelGGL(flux_finalize_kernel, dim3(1), dim3(256), 0, st, part, nt, c);
    return hipGetLastError();
}

hipError_t launch_commit(hipStream_t st, long n, double2 *g, const double2 *gn, const StepCtl *c) {
    hipLaunchKernelGGL(commit_kernel, vgrid(n), dim3(256), 0, st, n, g, gn, c);
    return hipGetLastError();
}

hipError_t launch_precond_rhs(hipStream_t st, long n, const double2 *g, const double2 *gn,
                              double2 *y, double2 *x, const StepCtl *c) {
    hipLaunchKernelGGL(precond_rhs_kernel, vgrid(n), dim3(256), 0, st, n, g, gn, y, x, c);
    return hipGetLastError();
}

hipError_t launch_precond_update(hipStream_t st, long n, double2 *g, const double2 *x,
                                 double *part, const StepCtl *c, const GmresCtl *gc) {
    hipLaunchKernelGGL(precond_update_kernel, vgrid(n), dim3(256), 0, st, n, g, x, part, c, gc);
    hipLaunchKernelGGL(precond_finalize_kernel, dim3(1), dim3(256), 0, st, part,
                       (int)((n + 255) / 256), (StepCtl *)c, gc);
    return hipGetLastError();
}
