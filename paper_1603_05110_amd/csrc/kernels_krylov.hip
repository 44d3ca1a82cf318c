// BiCGStab for the preconditioner solve P x = y, P = I - L_h (Section 4.2
// names GMRES or BiCGStab for it), with every scalar kept on the device.
// The iteration is van der Vorst's (1992) without preconditioning, x0 = 0 and
// the shadow residual equal to the first residual:
//   rho = (rh, r), beta = (rho / rho_old)(alpha / omega)
//   p = r + beta (p - omega v),   v = P p,   alpha = rho / (rh, v)
//   s = r - alpha v,               t = P s,   omega = (t, s) / (t, t)
//   x = x + alpha p + omega s,     r = s - omega t
// with the complex inner product conjugate-linear in its first argument.
// The control block is the GMRES one (done / conv / finished / bad / total),
// so the preconditioned update that follows reads it unchanged.  Every
// kernel returns at once when the solve is done or (sc given) when the
// Schwarz iteration is not at its preconditioned update, so chunks of
// iterations can be enqueued ahead of the host's check.  The vector kernels
// and the partial dot products are HBM-bound streams; the products with P
// are the L_h matvec kernels of the GMRES path.
#include "step_bodies.h"

namespace {

constexpr int KB = 256;   // blocks of the partial dot products

__device__ __forceinline__ bool sc_idle(const StepCtl *sc) {
    return sc && (sc->r_done != 1 || sc->k_done || sc->bad);
}

// conj(a) b
__device__ __forceinline__ double2 cdot1(double2 a, double2 b) {
    return cd(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return cd((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// r = rh = y, p = v = 0, x = 0
__global__ void bicg_init_kernel(long n, const double2 *y, double2 *x, double2 *r, double2 *rh,
                                 double2 *p, double2 *v, const StepCtl *sc) {
    if (sc_idle(sc)) return;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double2 z = cd(0.0, 0.0), yv = y[e];
    r[e] = yv;
    rh[e] = yv;
    p[e] = z;
    v[e] = z;
    x[e] = z;
}

// Block partials of (a1, b1) and (a2, b2) (a2 may be null), 4 doubles per
// block.  start = 1: the first dot of a solve, run while ctl->done is still
// set from the reset.
__global__ __launch_bounds__(256) void bicg_dot_kernel(long n, const double2 *a1, const double2 *b1,
                                                       const double2 *a2, const double2 *b2,
                                                       double *part, const GmresCtl *ctl,
                                                       const StepCtl *sc, int start) {
    if (sc_idle(sc) || (!start && ctl->done)) return;
    __shared__ double red[16];
    const long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long lo = (long)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        const double2 d = cdot1(a1[e], b1[e]);
        s0 += d.x;
        s1 += d.y;
        if (a2) {
            const double2 f = cdot1(a2[e], b2[e]);
            s2 += f.x;
            s3 += f.y;
        }
    }
    s0 = ctl_block_sum(s0, red);
    s1 = ctl_block_sum(s1, red);
    s2 = ctl_block_sum(s2, red);
    s3 = ctl_block_sum(s3, red);
    if (threadIdx.x == 0) {
        double *o = part + 4 * (long)blockIdx.x;
        o[0] = s0; o[1] = s1; o[2] = s2; o[3] = s3;
    }
}

// Reduces the block partials (fixed order) and applies one scalar step:
// phase 0 start (||y||), 1 rho and beta, 2 alpha, 3 omega, 4 ||r|| and the
// convergence test.
__global__ __launch_bounds__(256) void bicg_scalar_kernel(const double *part, int nb, int phase,
                                                          BicgState *S, GmresCtl *ctl,
                                                          const StepCtl *sc, int max_it) {
    if (sc_idle(sc) || (phase != 0 && ctl->done)) return;
    __shared__ double red[16];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        s0 += part[4 * b]; s1 += part[4 * b + 1]; s2 += part[4 * b + 2]; s3 += part[4 * b + 3];
    }
    s0 = ctl_block_sum(s0, red);
    s1 = ctl_block_sum(s1, red);
    s2 = ctl_block_sum(s2, red);
    s3 = ctl_block_sum(s3, red);
    if (threadIdx.x != 0) return;
    const double2 d1 = cd(s0, s1), d2 = cd(s2, s3);
    if (phase == 0) {
        const double bn = sqrt(fmax(d1.x, 0.0));
        ctl->done = 0; ctl->conv = 0; ctl->finished = 0; ctl->j = 0; ctl->total = 0;
        ctl->bnorm = bn;
        ctl->resid = bn;
        S->rho = cd(1.0, 0.0);
        S->alpha = cd(1.0, 0.0);
        S->omega = cd(1.0, 0.0);
        if (!isfinite(bn)) { ctl->bad = 1; ctl->done = 1; ctl->finished = 1; return; }
        if (bn == 0.0) { ctl->done = 1; ctl->finished = 1; ctl->conv = 1; }
        return;
    }
    if (phase == 1) {
        // rho = 0 or (after a vanishing omega) no progress: breakdown
        if (!(d1.x * d1.x + d1.y * d1.y > 0.0) || !isfinite(d1.x) || !isfinite(d1.y) ||
            !(S->omega.x * S->omega.x + S->omega.y * S->omega.y > 0.0)) {
            ctl->bad = 1; ctl->done = 1; ctl->finished = 1;
            return;
        }
        S->beta = cmul(cdiv(d1, S->rho), cdiv(S->alpha, S->omega));
        S->rho = d1;
        return;
    }
    if (phase == 2) {
        if (!(d1.x * d1.x + d1.y * d1.y > 0.0)) { ctl->bad = 1; ctl->done = 1; ctl->finished = 1; return; }
        S->alpha = cdiv(S->rho, d1);
        return;
    }
    if (phase == 3) {
        // omega = (t, s) / (t, t); t = 0 means s = 0: x is then exact
        S->omega = d2.x > 0.0 ? cscale(1.0 / d2.x, d1) : cd(0.0, 0.0);
        return;
    }
    const double rn = sqrt(fmax(d1.x, 0.0));
    ctl->total += 1;
    ctl->j += 1;
    ctl->resid = rn;
    if (!isfinite(rn)) { ctl->bad = 1; ctl->done = 1; ctl->finished = 1; return; }
    if (rn <= ctl->tol * ctl->bnorm) {
        ctl->done = 1; ctl->finished = 1; ctl->conv = 1;
    } else if (ctl->total >= max_it) {
        ctl->done = 1; ctl->finished = 1;
    }
}

// p = r + beta (p - omega v)
__global__ void bicg_p_kernel(long n, const double2 *r, const double2 *v, double2 *p,
                              const BicgState *S, const GmresCtl *ctl, const StepCtl *sc) {
    if (sc_idle(sc) || ctl->done) return;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    p[e] = cadd(r[e], cmul(S->beta, csub(p[e], cmul(S->omega, v[e]))));
}

// s = r - alpha v
__global__ void bicg_s_kernel(long n, const double2 *r, const double2 *v, double2 *s,
                              const BicgState *S, const GmresCtl *ctl, const StepCtl *sc) {
    if (sc_idle(sc) || ctl->done) return;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    s[e] = csub(r[e], cmul(S->alpha, v[e]));
}

// x = x + alpha p + omega s, r = s - omega t
__global__ void bicg_xr_kernel(long n, const double2 *p, const double2 *s, const double2 *t,
                               double2 *x, double2 *r, const BicgState *S, const GmresCtl *ctl,
                               const StepCtl *sc) {
    if (sc_idle(sc) || ctl->done) return;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double2 sv = s[e];
    x[e] = cadd(x[e], cadd(cmul(S->alpha, p[e]), cmul(S->omega, sv)));
    r[e] = csub(sv, cmul(S->omega, t[e]));
}

inline dim3 vgrid(long n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t launch_bicg_start(hipStream_t st, long n, const double2 *y, double2 *x, double2 *V,
                             double *part, BicgState *S, GmresCtl *ctl, const StepCtl *sc) {
    double2 *r = V, *rh = V + n, *p = V + 2 * n, *v = V + 3 * n;
    hipLaunchKernelGGL(bicg_init_kernel, vgrid(n), dim3(256), 0, st, n, y, x, r, rh, p, v, sc);
    hipLaunchKernelGGL(bicg_dot_kernel, dim3(KB), dim3(256), 0, st, n, y, y,
                       (const double2 *)nullptr, (const double2 *)nullptr, part, ctl, sc, 1);
    hipLaunchKernelGGL(bicg_scalar_kernel, dim3(1), dim3(256), 0, st, part, KB, 0, S, ctl, sc, 0);
    return hipGetLastError();
}

hipError_t launch_bicg_iteration(hipStream_t st, const Phys &P, const StripMeta *strips, int ncls,
                                 const LhPlan &pl, const double2 *LH, long n, double2 *V,
                                 double2 *x, double *part, BicgState *S, GmresCtl *ctl,
                                 const StepCtl *sc, int max_it) {
    double2 *r = V, *rh = V + n, *p = V + 2 * n, *v = V + 3 * n, *s = V + 4 * n, *t = V + 5 * n;
    const dim3 g = vgrid(n), b(256);
    hipLaunchKernelGGL(bicg_dot_kernel, dim3(KB), b, 0, st, n, rh, r, (const double2 *)nullptr,
                       (const double2 *)nullptr, part, ctl, sc, 0);
    hipLaunchKernelGGL(bicg_scalar_kernel, dim3(1), b, 0, st, part, KB, 1, S, ctl, sc, max_it);
    hipLaunchKernelGGL(bicg_p_kernel, g, b, 0, st, n, r, v, p, S, ctl, sc);
    hipError_t e = launch_lh_matvec(st, P, strips, ncls, pl, LH, p, v, 1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bicg_dot_kernel, dim3(KB), b, 0, st, n, rh, v, (const double2 *)nullptr,
                       (const double2 *)nullptr, part, ctl, sc, 0);
    hipLaunchKernelGGL(bicg_scalar_kernel, dim3(1), b, 0, st, part, KB, 2, S, ctl, sc, max_it);
    hipLaunchKernelGGL(bicg_s_kernel, g, b, 0, st, n, r, v, s, S, ctl, sc);
    e = launch_lh_matvec(st, P, strips, ncls, pl, LH, s, t, 1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bicg_dot_kernel, dim3(KB), b, 0, st, n, t, s, t, t, part, ctl, sc, 0);
    hipLaunchKernelGGL(bicg_scalar_kernel, dim3(1), b, 0, st, part, KB, 3, S, ctl, sc, max_it);
    hipLaunchKernelGGL(bicg_xr_kernel, g, b, 0, st, n, p, s, t, x, r, S, ctl, sc);
    hipLaunchKernelGGL(bicg_dot_kernel, dim3(KB), b, 0, st, n, r, r, (const double2 *)nullptr,
                       (const double2 *)nullptr, part, ctl, sc, 0);
    hipLaunchKernelGGL(bicg_scalar_kernel, dim3(1), b, 0, st, part, KB, 4, S, ctl, sc, max_it);
    return hipGetLastError();
}

int bicg_partials() { return 4 * KB; }
