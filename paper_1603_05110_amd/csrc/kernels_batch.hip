// Time-step kernels of a batch of independent instances (uneven meshes and
// strip layouts).  Each kernel covers every instance in one launch: the
// instance index comes from the grid, its mesh constants and buffers from
// the instance table, and the arithmetic is the same per-node / per-line body
// as the single-instance kernels.  Every kernel first reads the instance's
// step control and returns when that instance's phase is complete, so a
// fixed sequence of launches (a captured graph) can be replayed until every
// instance has converged.
#include "step_bodies.h"

namespace {

__global__ void b_check_finite_kernel(const InstDesc *tab) {
    const InstDesc &I = tab[blockIdx.y];
    long n = (long)I.P.nglob * I.P.ny;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long stride = (long)gridDim.x * blockDim.x;
    int bad = 0;
    for (; i < n; i += stride) {
        double2 v = I.u[i];
        if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
    }
    if (bad) atomicOr(I.flag, 1);
}

__global__ void b_zero_flags_kernel(const InstDesc *tab, int nb) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) *tab[b].flag = 0;
}

__global__ void b_mass_kernel(const InstDesc *tab) {
    const InstDesc &I = tab[blockIdx.y];
    const Phys P = I.P;
    if ((int)blockIdx.x >= P.nglob) return;
    mass_line(P, I.u, I.mass_part, blockIdx.x);
}

__global__ void b_mass_sum_kernel(const InstDesc *tab, int slot) {
    const InstDesc &I = tab[blockIdx.x];
    sum_block(I.mass_part, I.P.nglob, 1, I.scal + slot);
}

__global__ void b_step_init_kernel(const InstDesc *tab, StepCfg cfg) {
    if (threadIdx.x != 0) return;
    step_init_body(tab[blockIdx.x].ctl, cfg);
}

// guarded = 0: copy unconditionally (start of the step).  guarded = 1: the
// fixed point of a new Schwarz iteration restarts from u_{n-1} (no warm
// start): copy only for instances that have just begun iteration k > 1.
__global__ void b_copy_u_kernel(const InstDesc *tab, int guarded) {
    const InstDesc &I = tab[blockIdx.z];
    const Phys P = I.P;
    int L = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= P.lt || a >= P.ny) return;
    if (guarded) {
        const StepCtl *c = I.ctl;
        if (c->k_done || c->bad || c->k == 0 || c->q_iter != 0 || c->q_conv) return;
    }
    copy_u_at(P, I.strips, I.line_strip, I.u, I.zeta, L, a);
}

// A new Schwarz iteration starts only where the previous one has committed
// (ready), so replaying this launch mid-iteration changes nothing.
__global__ void b_iter_reset_kernel(const InstDesc *tab) {
    if (threadIdx.x != 0) return;
    StepCtl *c = tab[blockIdx.x].ctl;
    if (c->k_done || c->bad || !c->ready) return;
    iter_reset_body(c, tab[blockIdx.x].gctl);
}

__global__ __launch_bounds__(256) void b_residual_kernel(const InstDesc *tab) {
    const InstDesc &I = tab[blockIdx.z];
    const Phys P = I.P;
    int L = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= P.lt || a >= P.ny) return;
    if (fp_idle(I.ctl)) return;
    I.res[(long)L * P.ny + a] = residual_at(P, I.strips, I.line_strip, I.W, I.u, I.zeta, I.g, L, a);
}

__global__ void b_update_norms_kernel(const InstDesc *tab) {
    const InstDesc &I = tab[blockIdx.y];
    if ((int)blockIdx.x >= I.P.lt) return;
    if (fp_idle(I.ctl)) return;
    update_norms_line(I.P.ny, I.zeta, I.delta, I.line_part, blockIdx.x);
}

__global__ void b_q_check_kernel(const InstDesc *tab) {
    const InstDesc &I = tab[blockIdx.x];
    if (fp_idle(I.ctl)) return;
    q_check_block(I.P, I.strips, I.line_part, I.ctl);
}

__global__ void b_flux_kernel(const InstDesc *tab) {
    const InstDesc &I = tab[blockIdx.y];
    const StepCtl *c = I.ctl;
    if ((int)blockIdx.x >= 2 * (I.P.nsub - 1)) return;
    if (!c->q_conv || c->r_done || c->k_done || c->bad) return;
    flux_trace(I.P, I.strips, I.g, I.zeta, I.gn, I.trace_part, blockIdx.x);
}

__global__ void b_flux_finalize_kernel(const InstDesc *tab) {
    const InstDesc &I = tab[blockIdx.x];
    StepCtl *c = I.ctl;
    if (!c->q_conv || c->r_done || c->k_done || c->bad) return;
    flux_finalize_block(I.trace_part, 2 * (I.P.nsub - 1), c);
}

// g <- R(g) where the Schwarz map of this iteration has just been evaluated
// (commit set and not yet consumed).
__global__ void b_commit_kernel(const InstDesc *tab) {
    const InstDesc &I = tab[blockIdx.y];
    const StepCtl *c = I.ctl;
    if (!c->commit) return;
    long n = 2L * (I.P.nsub - 1) * I.P.ny;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) I.g[e] = I.gn[e];
}

__global__ void b_time_update_kernel(const InstDesc *tab) {
    const InstDesc &I = tab[blockIdx.z];
    const Phys P = I.P;
    int gl = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (gl >= P.nglob || a >= P.ny) return;
    time_update_at(P, I.gmap, I.zeta, I.u, gl, a);
}

}  // namespace

static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_b_check_finite(hipStream_t st, const InstDesc *tab, const BatchDims &d) {
    hipLaunchKernelGGL(b_zero_flags_kernel, dim3(cdiv(d.nb, 64)), dim3(64), 0, st, tab, d.nb);
    long n = (long)d.max_nglob * d.max_ny;
    unsigned blocks = cdiv(n, 256);
    if (blocks > 1024u) blocks = 1024u;
    hipLaunchKernelGGL(b_check_finite_kernel, dim3(blocks, d.nb), dim3(256), 0, st, tab);
    return hipGetLastError();
}

hipError_t launch_b_mass(hipStream_t st, const InstDesc *tab, const BatchDims &d, int slot) {
    hipLaunchKernelGGL(b_mass_kernel, dim3(d.max_nglob, d.nb), dim3(256), 0, st, tab);
    hipLaunchKernelGGL(b_mass_sum_kernel, dim3(d.nb), dim3(256), 0, st, tab, slot);
    return hipGetLastError();
}

hipError_t launch_b_step_init(hipStream_t st, const InstDesc *tab, const BatchDims &d,
                              const StepCfg &cfg) {
    hipLaunchKernelGGL(b_step_init_kernel, dim3(d.nb), dim3(64), 0, st, tab, cfg);
    return hipGetLastError();
}

hipError_t launch_b_copy_u(hipStream_t st, const InstDesc *tab, const BatchDims &d, int guarded) {
    hipLaunchKernelGGL(b_copy_u_kernel, dim3(cdiv(d.max_ny, 256), d.max_lt, d.nb), dim3(256), 0,
                       st, tab, guarded);
    return hipGetLastError();
}

hipError_t launch_b_iter_reset(hipStream_t st, const InstDesc *tab, const BatchDims &d) {
    hipLaunchKernelGGL(b_iter_reset_kernel, dim3(d.nb), dim3(64), 0, st, tab);
    return hipGetLastError();
}

hipError_t launch_b_residual(hipStream_t st, const InstDesc *tab, const BatchDims &d) {
    hipLaunchKernelGGL(b_residual_kernel, dim3(cdiv(d.max_ny, 256), d.max_lt, d.nb), dim3(256), 0,
                       st, tab);
    return hipGetLastError();
}

hipError_t launch_b_update_norms(hipStream_t st, const InstDesc *tab, const BatchDims &d) {
    hipLaunchKernelGGL(b_update_norms_kernel, dim3(d.max_lt, d.nb), dim3(256), 0, st, tab);
    return hipGetLastError();
}

hipError_t launch_b_q_check(hipStream_t st, const InstDesc *tab, const BatchDims &d) {
    hipLaunchKernelGGL(b_q_check_kernel, dim3(d.nb), dim3(256), 0, st, tab);
    return hipGetLastError();
}

hipError_t launch_b_flux(hipStream_t st, const InstDesc *tab, const BatchDims &d) {
    hipLaunchKernelGGL(b_flux_kernel, dim3(d.max_ntr, d.nb), dim3(256), 0, st, tab);
    hipLaunchKernelGGL(b_flux_finalize_kernel, dim3(d.nb), dim3(256), 0, st, tab);
    return hipGetLastError();
}

hipError_t launch_b_commit(hipStream_t st, const InstDesc *tab, const BatchDims &d) {
    hipLaunchKernelGGL(b_commit_kernel, dim3(cdiv(d.max_ng, 256), d.nb), dim3(256), 0, st, tab);
    return hipGetLastError();
}

hipError_t launch_b_time_update(hipStream_t st, const InstDesc *tab, const BatchDims &d) {
    hipLaunchKernelGGL(b_time_update_kernel, dim3(cdiv(d.max_ny, 256), d.max_nglob, d.nb),
                       dim3(256), 0, st, tab);
    return hipGetLastError();
}
