// Q1 stencil kernels on x-strips (Section 2.2, eq. NproblemRobinNL):
// coefficient assembly of the strip operator, the fixed-point residual, the
// flux update of the interface vector (eq. fluxlr), the time update and the
// discrete mass.  All FP64; memory-bound, one thread per node.
#include "osm_internal.h"

namespace {

// Integrals between node (i,a) and node (ip,b) of one strip with nx lines:
// mass m, stiffness s, potential-weighted mass w = int phi_h psi psi (phi
// replaced by its Q1 interpolant, triple products exact) and the y-mass of
// the left/right edge lines (boundary mass M^Gamma).  Elements of the strip
// only: a strip is its own finite-element domain.
struct KParts {
    double m, s, w, edge_l, edge_r;
};

template <class PhiF>
__device__ __forceinline__ KParts kparts(int i, int a, int ip, int b, int nx, int ny,
                                         double hx, double hy, PhiF phi) {
    KParts k = {0.0, 0.0, 0.0, 0.0, 0.0};
    int exlo = max(max(i, ip) - 1, 0), exhi = min(min(i, ip), nx - 2);
    int eylo = max(max(a, b) - 1, 0), eyhi = min(min(a, b), ny - 2);
    for (int ex = exlo; ex <= exhi; ++ex) {
        int Ax = i - ex, Bx = ip - ex;
        double mx = hx * ref_mass(Ax, Bx), sx = ref_stiff(Ax, Bx) / hx;
        for (int ey = eylo; ey <= eyhi; ++ey) {
            int Ay = a - ey, By = b - ey;
            double my = hy * ref_mass(Ay, By), sy = ref_stiff(Ay, By) / hy;
            k.m += mx * my;
            k.s += sx * my + mx * sy;
            double acc = 0.0;
#pragma unroll
            for (int cx = 0; cx < 2; ++cx)
#pragma unroll
                for (int cy = 0; cy < 2; ++cy)
                    acc += phi(ex + cx, ey + cy) * ref_triple(cx, Ax, Bx) * ref_triple(cy, Ay, By);
            k.w += hx * hy * acc;
        }
    }
    if (i == ip && (i == 0 || i == nx - 1)) {
        double my = 0.0;
        for (int ey = eylo; ey <= eyhi; ++ey) my += hy * ref_mass(a - ey, b - ey);
        if (i == 0) k.edge_l = my;
        if (i == nx - 1) k.edge_r = my;
    }
    return k;
}

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
            dv = cd(-P.c * k.s + k.w, (2.0 / P.dt) * k.m + P.c * (s.pl * k.edge_l + s.pr * k.edge_r));
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
__global__ void residual_kernel(Phys P, const StripMeta *strips, const int *line_strip,
                                const double *W, const double2 *u_old, const double2 *zeta,
                                const double2 *g, double2 *res, const StepCtl *c) {
    if (c && (c->q_conv || c->k_done || c->bad)) return;
    int L = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    int ny = P.ny;
    if (a >= ny) return;
    int j = line_strip[L];
    StripMeta s = strips[j];
    int i = L - s.off;
    const double *Wl = W + (long)s.line0 * ny;
    const double2 *ul = u_old + (long)s.line0 * ny;
    const double2 *zl = zeta + (long)s.off * ny;
    double beta = P.beta;
    auto phi = [&](int ii, int kk) -> double {
        double2 z = zl[(long)ii * ny + kk];
        return Wl[(long)ii * ny + kk] + beta * (z.x * z.x + z.y * z.y);
    };
    double2 acc = cd(0.0, 0.0);
    const double2 *trace = nullptr;
    if (i == 0 && j >= 1) trace = g + (long)(2 * (j - 1) + 1) * ny;             // l_j
    if (i == s.nx - 1 && j <= P.nsub - 2) trace = g + (long)(2 * j) * ny;       // r_j
    for (int ip = max(i - 1, 0); ip <= min(i + 1, s.nx - 1); ++ip) {
        for (int b = max(a - 1, 0); b <= min(a + 1, ny - 1); ++b) {
            KParts k = kparts(i, a, ip, b, s.nx, ny, P.hx, P.hy, phi);
            double2 z = zl[(long)ip * ny + b];
            double2 u = ul[(long)ip * ny + b];
            // 2i/dt m (u - z)
            double2 du = csub(u, z);
            acc.x += -(2.0 / P.dt) * k.m * du.y;
            acc.y += (2.0 / P.dt) * k.m * du.x;
            // + c s z - w z
            double cs = P.c * k.s - k.w;
            acc.x += cs * z.x;
            acc.y += cs * z.y;
            // - i c (pl edge_l + pr edge_r) z
            double e = P.c * (s.pl * k.edge_l + s.pr * k.edge_r);
            acc.x += e * z.y;
            acc.y += -e * z.x;
            // - c M^Gamma trace
            if (trace && ip == i) {
                double my = (i == 0) ? k.edge_l : k.edge_r;
                double2 t = trace[b];
                acc.x -= P.c * my * t.x;
                acc.y -= P.c * my * t.y;
            }
        }
    }
    res[(long)L * ny + a] = acc;
}

__global__ void copy_u_kernel(Phys P, const StripMeta *strips, const int *line_strip,
                              const double2 *u, double2 *zeta) {
    int L = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= P.ny) return;
    StripMeta s = strips[line_strip[L]];
    int gl = s.line0 + (L - s.off);
    zeta[(long)L * P.ny + a] = u[(long)gl * P.ny + a];
}

// zeta += delta on one packed line; per-line partial sums |delta|^2, |zeta|^2
// and a non-finite counter.
__global__ void update_norms_kernel(Phys P, double2 *zeta, const double2 *delta, double *part,
                                    const StepCtl *c) {
    if (c && (c->q_conv || c->k_done || c->bad)) return;
    int L = blockIdx.x;
    int ny = P.ny;
    double s_d = 0.0, s_z = 0.0, bad = 0.0;
    for (int a = threadIdx.x; a < ny; a += blockDim.x) {
        long o = (long)L * ny + a;
        double2 d = delta[o];
        double2 z = cadd(zeta[o], d);
        zeta[o] = z;
        s_d += d.x * d.x + d.y * d.y;
        s_z += z.x * z.x + z.y * z.y;
        if (!isfinite(d.x) || !isfinite(d.y)) bad += 1.0;
    }
    __shared__ double red[3][256];
    red[0][threadIdx.x] = s_d;
    red[1][threadIdx.x] = s_z;
    red[2][threadIdx.x] = bad;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
            red[2][threadIdx.x] += red[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * L] = red[0][0];
        part[3 * L + 1] = red[1][0];
        part[3 * L + 2] = red[2][0];
    }
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

// Flux update, eq. fluxlr with S = -ip (Jacobi):
//   new r_i     = -l_{i+1} - 2ip v_{i+1}(first line)
//   new l_{i+1} = -r_i     - 2ip v_i(last line)
// Per-trace partial sums of |gn - g|^2 and |gn|^2.
__global__ void flux_kernel(Phys P, const StripMeta *strips, const double2 *g,
                            const double2 *v, double2 *gn, double *part, const StepCtl *c) {
    if (c && (!c->q_conv || c->r_done || c->k_done || c->bad)) return;
    int t = blockIdx.x;           // trace 0 .. 2(N-1)-1
    int ny = P.ny;
    int i = t >> 1;
    const double2 *src;
    const double2 *vt;
    if ((t & 1) == 0) {           // r_i from strip i+1's left line
        src = g + (long)(2 * i + 1) * ny;
        vt = v + (long)strips[i + 1].off * ny;
    } else {                      // l_{i+1} from strip i's right line
        src = g + (long)(2 * i) * ny;
        StripMeta s = strips[i];
        vt = v + (long)(s.off + s.nx - 1) * ny;
    }
    double tp = 2.0 * P.p;
    double sd = 0.0, sn = 0.0;
    for (int a = threadIdx.x; a < ny; a += blockDim.x) {
        double2 x = src[a], w = vt[a];
        // -x - 2ip w = (-x.re + 2p w.im) + i(-x.im - 2p w.re)
        double2 r = cd(-x.x + tp * w.y, -x.y - tp * w.x);
        double2 o = g[(long)t * ny + a];
        gn[(long)t * ny + a] = r;
        sd += (r.x - o.x) * (r.x - o.x) + (r.y - o.y) * (r.y - o.y);
        sn += r.x * r.x + r.y * r.y;
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = sd;
    red[1][threadIdx.x] = sn;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * t] = red[0][0];
        part[2 * t + 1] = red[1][0];
    }
}

// u_n = 2 vbar - u_{n-1} on every global node; vbar is the strip value, the
// mean of the two copies on an interface line.
__global__ void time_update_kernel(Phys P, const int2 *gmap, const double2 *v, double2 *u) {
    int gl = blockIdx.y;
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    int ny = P.ny;
    if (a >= ny) return;
    int2 m = gmap[gl];
    double2 vb = v[(long)m.x * ny + a];
    if (m.y >= 0) vb = cscale(0.5, cadd(vb, v[(long)m.y * ny + a]));
    long o = (long)gl * ny + a;
    double2 uo = u[o];
    u[o] = cd(2.0 * vb.x - uo.x, 2.0 * vb.y - uo.y);
}

// Per-line partials of u* M u with the global Q1 mass M = M1x (x) M1y.
__global__ void mass_kernel(Phys P, const double2 *u, double *part) {
    int gl = blockIdx.x;
    int ny = P.ny, ng = P.nglob;
    double hx = P.hx, hy = P.hy;
    double acc = 0.0;
    for (int a = threadIdx.x; a < ny; a += blockDim.x) {
        double2 mu = cd(0.0, 0.0);
        for (int ip = max(gl - 1, 0); ip <= min(gl + 1, ng - 1); ++ip) {
            double mx;
            if (ip != gl) mx = hx / 6.0;
            else mx = (gl == 0 || gl == ng - 1) ? hx / 3.0 : 2.0 * hx / 3.0;
            for (int b = max(a - 1, 0); b <= min(a + 1, ny - 1); ++b) {
                double my;
                if (b != a) my = hy / 6.0;
                else my = (a == 0 || a == ny - 1) ? hy / 3.0 : 2.0 * hy / 3.0;
                double2 x = u[(long)ip * ny + b];
                mu.x += mx * my * x.x;
                mu.y += mx * my * x.y;
            }
        }
        double2 x = u[(long)gl * ny + a];
        acc += x.x * mu.x + x.y * mu.y;   // Re(conj(x) * mu)
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[gl] = red[0];
}

// Deterministic sum of n strided values (one block).
__global__ void sum_kernel(const double *part, int n, int stride, double *out) {
    __shared__ double red[256];
    for (int c = 0; c < stride; ++c) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[(long)i * stride + c];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = red[0];
        __syncthreads();
    }
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

}  // namespace

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
                           const StepCtl *c) {
    hipLaunchKernelGGL(residual_kernel, node_grid(P.ny, P.lt), dim3(256), 0, st, P, strips,
                       line_strip, W, u_old, zeta, g, res, c);
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
                       const StepCtl *c) {
    hipLaunchKernelGGL(flux_kernel, dim3(2 * (P.nsub - 1)), dim3(256), 0, st, P, strips, g, v,
                       gn, part, c);
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
