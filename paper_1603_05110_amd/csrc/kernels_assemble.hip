// Q1 stencil kernels on x-strips (Section 2.2, eq. NproblemRobinNL):
// coefficient assembly of the strip operator, the fixed-point residual, the
// flux update of the interface vector (eq. fluxlr), the time update and the
// discrete mass.  All FP64; memory-bound, one thread per node.
#include "step_bodies.h"

namespace {

// D_i (diagonal block, line i with itself) and U_i (line i with line i+1) of
// K_j(W) = 2i/dt M - c S + M_W + i c (pl M^Gamma_l + pr M^Gamma_r), stored as
// 3 complex diagonals per row: [row][d] = K(row, row + d - 1).
__global__ void coef_kernel(Phys P, const StripMeta *strips, const int *line_strip,
                            const double *W, int w_is_zero, double2 *Dc, double2 *Uc,
                            int line_begin) {
    int L = line_begin + blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    int ny = P.ny;
    if (a >= ny) return;
    StripMeta s = strips[line_strip[L]];
    int i = L - s.off;
    const double *Wl = W + (long)s.line0 * ny;
    auto phi = [&](int ii, int kk) -> double { return w_is_zero ? 0.0 : Wl[(long)ii * ny + kk]; };
    long o = ((long)(L - line_begin) * ny + a) * 3;
    for (int d = 0; d < 3; ++d) {
        int b = a + d - 1;
        double2 dv = cd(0.0, 0.0), uv = cd(0.0, 0.0);
        if (b >= 0 && b < ny) {
            KParts k = kparts(i, a, i, b, s.nx, ny, P.hx, P.hy, phi);
            // + i c (pl + i pl_im) M^Gamma_l + i c (pr + i pr_im) M^Gamma_r
            dv = cd(-P.c * k.s + k.w - P.c * (s.pl_im * k.edge_l + s.pr_im * k.edge_r),
                    (2.0 / P.dt) * k.m + P.c * (s.pl * k.edge_l + s.pr * k.edge_r));
            if (i + 1 < s.nx) {
                KParts ku = kparts(i, a, i + 1, b, s.nx, ny, P.hx, P.hy, phi);
                uv = cd(-P.c * ku.s + ku.w, (2.0 / P.dt) * ku.m);
            }
        }
        Dc[o + d] = dv;
        Uc[o + d] = uv;
    }
}

// Fixed-point residual of one strip node (residual form of the fixed point
// with the nonlinearity on the right-hand side):
//   res = 2i/dt M_j u_{j,n-1} - c M^Gamma Q^T (l_j; r_j) - K_j(W + beta|zeta|^2) zeta.
// With the factor of K_j(W), zeta + K_j(W)^{-1} res equals
// K_j(W)^{-1}(F - M_{beta|zeta|^2} zeta): the paper's fixed-point update.
__global__ __launch_bounds__(256) void residual_kernel(Phys P, const StripMeta *strips, const int *line_strip,
                                const double *W, const double2 *u_old, const double2 *zeta,
                                const double2 *g, double2 *res, const StepCtl *c,
                                const double2 *psi) {
    if (c && fp_idle(c)) return;
    int L = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= P.ny) return;
    res[(long)L * P.ny + a] = residual_at(P, strips, line_strip, W, u_old, zeta, g, L, a, psi);
}

__global__ void copy_u_kernel(Phys P, const StripMeta *strips, const int *line_strip,
                              const double2 *u, double2 *zeta) {
    int L = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= P.ny) return;
    copy_u_at(P, strips, line_strip, u, zeta, L, a);
}

// zeta += delta on one packed line, with the per-line partial norms.
__global__ void update_norms_kernel(Phys P, double2 *zeta, const double2 *delta, double *part,
                                    const StepCtl *c) {
    if (c && fp_idle(c)) return;
    update_norms_line(P.ny, zeta, delta, part, blockIdx.x);
}

__global__ void strip_sums_kernel(Phys P, const StripMeta *strips, const double *part,
                                  double *out) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P.nsub) return;
    StripMeta s = strips[j];
    double a = 0, b = 0, c = 0;
    for (int i = 0; i < s.nx; ++i) {
        a += part[3 * (s.off + i)];
        b += part[3 * (s.off + i) + 1];
        c += part[3 * (s.off + i) + 2];
    }
    out[3 * j] = a;
    out[3 * j + 1] = b;
    out[3 * j + 2] = c;
}

// Flux update of every trace (eq. fluxlr), per-trace partial norms.
__global__ void flux_kernel(Phys P, const StripMeta *strips, const double2 *g,
                            const double2 *v, double2 *gn, double *part, const StepCtl *c,
                            const double2 *psi) {
    if (c && (!c->q_conv || c->r_done || c->k_done || c->bad)) return;
    flux_trace(P, strips, g, v, gn, part, blockIdx.x, psi);
}

// u_n = 2 vbar - u_{n-1} on every global node.
__global__ void time_update_kernel(Phys P, const int2 *gmap, const double2 *v, double2 *u) {
    int gl = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= P.ny) return;
    time_update_at(P, gmap, v, u, gl, a);
}

// Per-line partials of u* M u.
__global__ void mass_kernel(Phys P, const double2 *u, double *part) {
    mass_line(P, u, part, blockIdx.x);
}

// Deterministic sum of n strided values (one block).
__global__ void sum_kernel(const double *part, int n, int stride, double *out) {
    sum_block(part, n, stride, out);
}

// W_n = (V_t(t1) + V_t(t0))/2 with V_t(t, x~) = V(A(t) x~),
// A(t) = [[cos wt, sin wt], [-sin wt, cos wt]], V = vxx x^2 + vyy y^2
// (Section 5.2.1, eqs. x1Ax and u1u; W_n as in Section 2.1).
__global__ void rotating_W_kernel(Phys P, double xl, double yb, double omega, double vxx,
                                  double vyy, double t1, double t0, double *W) {
    int gl = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= P.ny) return;
    double xt = xl + P.hx * gl, yt = yb + P.hy * a;
    double acc = 0.0;
    double ts[2] = {t1, t0};
    for (int q = 0; q < 2; ++q) {
        double c = cos(omega * ts[q]), s = sin(omega * ts[q]);
        double x = c * xt + s * yt, y = -s * xt + c * yt;
        acc += vxx * x * x + vyy * y * y;
    }
    W[(long)gl * P.ny + a] = 0.5 * acc;
}

__global__ void check_finite_kernel(const double2 *x, long n, int *flag) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long stride = (long)gridDim.x * blockDim.x;
    int bad = 0;
    for (; i < n; i += stride) {
        double2 v = x[i];
        if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
    }
    if (bad) atomicOr(flag, 1);
}

// Largest |b| (real and imaginary parts) of every packed line: one block
// per line.  The complex-FP32 solve turns the largest value of a strip into
// a power-of-two scale.
__device__ __forceinline__ void line_absmax_body(const double2 *b, int n, double *out) {
    double m = 0.0;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        double2 v = b[e];
        m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
    }
    __shared__ double red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void line_absmax_kernel(int ny, const double2 *b, double *lmax, const StepCtl *c) {
    if (c && fp_idle(c)) return;
    line_absmax_body(b + (long)blockIdx.x * ny, ny, lmax + blockIdx.x);
}

__global__ void b_line_absmax_kernel(const BStrip *strips, int guard) {
    const BStrip &s = strips[blockIdx.y];
    if ((int)blockIdx.x >= s.nx) return;
    if (guard && s.ctl && fp_idle(s.ctl)) return;
    line_absmax_body(s.b + (long)blockIdx.x * s.n, s.n, s.lmax + blockIdx.x);
}

}  // namespace

hipError_t launch_line_absmax(hipStream_t st, const Phys &P, const double2 *b, double *lmax,
                              const StepCtl *c) {
    hipLaunchKernelGGL(line_absmax_kernel, dim3(P.lt), dim3(256), 0, st, P.ny, b, lmax, c);
    return hipGetLastError();
}

hipError_t launch_b_line_absmax(hipStream_t st, const BStrip *strips, int nstrips, int max_nx,
                                int guard) {
    hipLaunchKernelGGL(b_line_absmax_kernel, dim3(max_nx, nstrips), dim3(256), 0, st, strips,
                       guard);
    return hipGetLastError();
}

static inline dim3 node_grid(int ny, int lines) { return dim3((ny + 255) / 256, lines); }

hipError_t launch_coef(hipStream_t st, const Phys &P, const StripMeta *strips,
                       const int *line_strip, const double *W, int w_is_zero,
                       double2 *Dc, double2 *Uc, int line_begin, int line_count) {
    hipLaunchKernelGGL(coef_kernel, node_grid(P.ny, line_count), dim3(256), 0, st, P, strips,
                       line_strip, W, w_is_zero, Dc, Uc, line_begin);
    return hipGetLastError();
}

hipError_t launch_residual(hipStream_t st, const Phys &P, const StripMeta *strips,
                           const int *line_strip, const double *W, const double2 *u_old,
                           const double2 *zeta, const double2 *g, double2 *res,
                           const StepCtl *c, const double2 *psi) {
    hipLaunchKernelGGL(residual_kernel, node_grid(P.ny, P.lt), dim3(256), 0, st, P, strips,
                       line_strip, W, u_old, zeta, g, res, c, psi);
    return hipGetLastError();
}

hipError_t launch_copy_u_to_strips(hipStream_t st, const Phys &P, const StripMeta *strips,
                                   const int *line_strip, const double2 *u, double2 *zeta) {
    hipLaunchKernelGGL(copy_u_kernel, node_grid(P.ny, P.lt), dim3(256), 0, st, P, strips,
                       line_strip, u, zeta);
    return hipGetLastError();
}

hipError_t launch_update_norms(hipStream_t st, const Phys &P, double2 *zeta,
                               const double2 *delta, double *line_part, const StepCtl *c) {
    hipLaunchKernelGGL(update_norms_kernel, dim3(P.lt), dim3(256), 0, st, P, zeta, delta,
                       line_part, c);
    return hipGetLastError();
}

hipError_t launch_strip_sums(hipStream_t st, const Phys &P, const StripMeta *strips,
                             const double *line_part, double *strip_out) {
    hipLaunchKernelGGL(strip_sums_kernel, dim3((P.nsub + 63) / 64), dim3(64), 0, st, P, strips,
                       line_part, strip_out);
    return hipGetLastError();
}

hipError_t launch_flux(hipStream_t st, const Phys &P, const StripMeta *strips,
                       const double2 *g, const double2 *v, double2 *gn, double *part,
                       const StepCtl *c, const double2 *psi) {
    hipLaunchKernelGGL(flux_kernel, dim3(2 * (P.nsub - 1)), dim3(256), 0, st, P, strips, g, v,
                       gn, part, c, psi);
    return hipGetLastError();
}

hipError_t launch_time_update(hipStream_t st, const Phys &P, const int2 *gline_map,
                              const double2 *v, double2 *u) {
    hipLaunchKernelGGL(time_update_kernel, node_grid(P.ny, P.nglob), dim3(256), 0, st, P,
                       gline_map, v, u);
    return hipGetLastError();
}

hipError_t launch_mass_partials(hipStream_t st, const Phys &P, const double2 *u, double *part) {
    hipLaunchKernelGGL(mass_kernel, dim3(P.nglob), dim3(256), 0, st, P, u, part);
    return hipGetLastError();
}

hipError_t launch_sum(hipStream_t st, const double *part, int n, int stride, double *out) {
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, part, n, stride, out);
    return hipGetLastError();
}

hipError_t launch_rotating_W(hipStream_t st, const Phys &P, double xl, double yb,
                             double omega, double vxx, double vyy, double t1, double t0,
                             double *W) {
    hipLaunchKernelGGL(rotating_W_kernel, node_grid(P.ny, P.nglob), dim3(256), 0, st, P, xl,
                       yb, omega, vxx, vyy, t1, t0, W);
    return hipGetLastError();
}

hipError_t launch_check_finite(hipStream_t st, const double2 *x, long n, int *flag) {
    long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, n, flag);
    return hipGetLastError();
}
