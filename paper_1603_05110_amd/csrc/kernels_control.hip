// Device-side control of one time step.  The decisions of the fixed point
// (Section 2.2: stop when the increment is small), of the Schwarz iteration
// (Section 5: stop when ||g^{k+1} - g^k|| < tol) and of the preconditioned
// update (eq. algo_pd) are taken by one-block kernels that write a StepCtl in
// device memory; every kernel of an iteration reads the flags first and
// returns at once when its phase is already complete.  The host can then
// enqueue a whole Schwarz iteration and synchronise once per iteration.
#include "step_bodies.h"

namespace {

__global__ void step_init_kernel(StepCtl *c, StepCfg cfg) {
    if (threadIdx.x != 0) return;
    step_init_body(c, cfg);
}

// Start of Schwarz iteration k (the host enqueues one per iteration).
__global__ void iter_reset_kernel(StepCtl *c, GmresCtl *g) {
    if (threadIdx.x != 0) return;
    if (c->k_done || c->bad) return;
    iter_reset_body(c, g);
}

__global__ void copy_u_guarded_kernel(Phys P, const StripMeta *strips, const int *line_strip,
                                      const double2 *u, double2 *zeta, const StepCtl *c) {
    if (c->k_done || c->bad) return;
    int L = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= P.ny) return;
    copy_u_at(P, strips, line_strip, u, zeta, L, a);
}

__global__ void q_check_kernel(Phys P, const StripMeta *strips, const double *part, StepCtl *c,
                               double *dprev) {
    if (c->q_conv || c->k_done || c->bad) return;
    q_check_block(P, strips, part, c, dprev);
}

__global__ void flux_finalize_kernel(const double *part, int nt, StepCtl *c) {
    if (!c->q_conv || c->r_done || c->k_done || c->bad) return;
    flux_finalize_block(part, nt, c);
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
    sx = ctl_block_sum(sx, red);
    sg = ctl_block_sum(sg, red);
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
    a = ctl_block_sum(a, red);
    b = ctl_block_sum(b, red);
    if (threadIdx.x != 0) return;
    double inc = sqrt(a), ref = sqrt(b);
    c->r_done = 2;
    c->ready = 1;                 // a batched replay may start the next iteration
    c->gm_total += gc->total;
    if (!isfinite(inc)) { c->bad = 1; return; }
    c->k += 1;
    c->inc = inc;
    c->ref = ref;
    c->prev_rel = inc / fmax(ref, 1e-300);
    if (c->k == 1) c->first_rel = c->prev_rel;
    double thr = c->cfg.tol_k_rel ? c->cfg.tol_k * fmax(ref, 1e-300) : c->cfg.tol_k;
    if (c->cfg.fixed_k > 0) { if (c->k >= c->cfg.fixed_k) c->k_done = 1; }
    else if (inc < thr) c->k_done = 1;
}

}  // namespace

static inline dim3 vgrid(long n) { return dim3((unsigned)((n + 255) / 256)); }

// Random first interface vector (Section 5, initial vectors).  SplitMix64
// (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
// 2014): state_j = seed + (j + 1) * 0x9E3779B97F4A7C15, output = the mix of
// state_j by two xor-shift-multiply rounds and a final xor-shift, so output
// j is computed on its own (counter-based); u(j) = (output >> 11) * 2^-53.
namespace {
__device__ __forceinline__ double splitmix_unit(uint64_t seed, uint64_t j) {
    uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

__global__ void random_interface_kernel(double2 *g, long n, uint64_t seed) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) g[k] = cd(splitmix_unit(seed, 2 * (uint64_t)k), splitmix_unit(seed, 2 * (uint64_t)k + 1));
}
}  // namespace

hipError_t launch_random_interface(hipStream_t st, double2 *g, long n, uint64_t seed) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(random_interface_kernel, vgrid(n), dim3(256), 0, st, g, n, seed);
    return hipGetLastError();
}

hipError_t launch_step_init(hipStream_t st, StepCtl *c, const StepCfg &cfg) {
    hipLaunchKernelGGL(step_init_kernel, dim3(1), dim3(64), 0, st, c, cfg);
    return hipGetLastError();
}

// one thread per 32-bit word of each structure; the stores go to pinned
// host memory and are visible to the host once the stream has synchronised
__global__ void ctl_gather_kernel(const StepCtl *s, const GmresCtl *g, const int *err,
                                  CtlMirror *out) {
    const int t = threadIdx.x;
    constexpr int ws = (int)(sizeof(StepCtl) / sizeof(int)), wg = (int)(sizeof(GmresCtl) / sizeof(int));
    static_assert(sizeof(StepCtl) % sizeof(int) == 0 && sizeof(GmresCtl) % sizeof(int) == 0,
                  "control structures are copied as 32-bit words");
    static_assert(ws + wg + 1 <= 256, "one thread per word");
    if (t < ws) reinterpret_cast<int *>(&out->s)[t] = reinterpret_cast<const int *>(s)[t];
    else if (t < ws + wg) {
        if (g) reinterpret_cast<int *>(&out->g)[t - ws] = reinterpret_cast<const int *>(g)[t - ws];
    } else if (t == ws + wg) {
        out->err = *err;
    }
}

hipError_t launch_ctl_gather(hipStream_t st, const StepCtl *s, const GmresCtl *g, const int *err,
                             CtlMirror *out) {
    hipLaunchKernelGGL(ctl_gather_kernel, dim3(1), dim3(256), 0, st, s, g, err, out);
    return hipGetLastError();
}

__global__ void scalar_gather_kernel(const int *flag, const double *val, CtlMirror *out) {
    if (threadIdx.x == 0) {
        if (flag) out->flag = *flag;
        out->val = *val;
    }
}

hipError_t launch_scalar_gather(hipStream_t st, const int *flag, const double *val,
                                CtlMirror *out) {
    hipLaunchKernelGGL(scalar_gather_kernel, dim3(1), dim3(64), 0, st, flag, val, out);
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
                          const double *part, StepCtl *c, double *dprev) {
    hipLaunchKernelGGL(q_check_kernel, dim3(1), dim3(1024), 0, st, P, strips, part, c, dprev);
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
