// The absorbing transmission condition S_pade^m (Section 2.1, eqs. TCS and
// TCS_phi; Section 2.2, eq. NproblemSPNL) on every strip edge.
//
// Each strip edge e carries m edge functions phi_{e,s} (ny values each) that
// solve the 1-D edge problem
//     D_{e,s} phi_{e,s} = M^G zeta_e - M^G_f phi_{e,s}^{prev},
//     D_{e,s} = (2i/dt + d_s) M^G - c S^G + M^G_W       (tridiagonal in y),
// and enter the strip equation through -sum_s B_s phi_{e,s} with
// B_s = -i c a_s d_s M^G.  Eliminating them (the Schur form the paper writes
// after eq. NproblemSPL) adds to the strip operator, on the edge line, the
// dense complex-symmetric block
//     E_e = -i c M^G G_e,      G_e = sum_s a_s d_s D_{e,s}^{-1} M^G,
// on top of the diagonal term i c (sum_s a_s) M^G.  The factor adds E_e to
// the Schur complement of each edge line before inverting it, so the strip
// solve is unchanged; the fixed point in residual form carries the edge
// functions as extra unknowns:
//   residual   r_phi = M^G zeta_e - (D_s + M^G_f) phi_s,  z_s = D_s^{-1} r_phi,
//              b_edge += i c M^G sum_s a_s d_s z_s          (eliminated rhs),
//   update     phi_s += z_s + D_s^{-1} M^G dzeta_e          (after the solve),
//              psi_e = sum_s a_s d_s phi_s,
// and the flux update uses S v = -i (sum a_s) v + i psi_e.
//
// Every tridiagonal edge system is solved by the Thomas algorithm from an LU
// factorisation kept per (edge, s) (sub-diagonal, modified super-diagonal,
// inverse pivots); D_{e,s} is complex symmetric with a positive-definite
// imaginary part (2/dt M^G + Im(d_s) M^G), so no pivoting is needed.
#include "step_bodies.h"

namespace {

// 1-D Q1 integrals along y on nodes a, b (|a - b| <= 1) of a line of ny
// nodes: mass, stiffness and the weighted mass with w interpolated linearly
// (triple products exact).
struct Line1D {
    double m, s, w;
};
template <class WF>
__device__ __forceinline__ Line1D line1d(int a, int b, int ny, double hy, WF wv) {
    Line1D r = {0.0, 0.0, 0.0};
    const int lo = max(max(a, b) - 1, 0), hi = min(min(a, b), ny - 2);
    for (int e = lo; e <= hi; ++e) {
        const int A = a - e, B = b - e;
        r.m += hy * ref_mass(A, B);
        r.s += ref_stiff(A, B) / hy;
        r.w += hy * (wv(e) * ref_triple(0, A, B) + wv(e + 1) * ref_triple(1, A, B));
    }
    return r;
}

// Global node-line of edge e (strip e / 2, side e % 2), or -1 for the free
// edge (W = 0) used by the L_h build.
__device__ __forceinline__ int edge_gline(const StripMeta *strips, int e, int nedge) {
    if (e >= nedge) return -1;
    const StripMeta s = strips[e >> 1];
    return (e & 1) ? s.line0 + s.nx - 1 : s.line0;
}
__device__ __forceinline__ int edge_pline(const StripMeta *strips, int e) {
    const StripMeta s = strips[e >> 1];
    return (e & 1) ? s.off + s.nx - 1 : s.off;
}

// LU factors of D_{e,s} for edges e < ne (ne = nedge, plus one free edge when
// with_free): thread per (e, s).
__global__ void pade_lu_kernel(Phys P, const StripMeta *strips, const double *W, int nedge,
                               int with_free, int e_first, int m, const double2 *ad,
                               double2 *sub, double2 *cp, double2 *inv) {
    const int t = e_first * m + blockIdx.x * blockDim.x + threadIdx.x;
    const int ne = nedge + (with_free ? 1 : 0);
    if (t >= ne * m) return;
    const int e = t / m, s = t % m;
    const int ny = P.ny, gl = edge_gline(strips, e, nedge);
    const double *Wl = gl >= 0 ? W + (long)gl * ny : nullptr;
    auto wv = [&](int k) -> double { return Wl ? Wl[k] : 0.0; };
    const double2 ds = ad[2 * s + 1];
    const long o = (long)t * ny;
    double2 prev_cp = cd(0.0, 0.0);
    for (int a = 0; a < ny; ++a) {
        // D(a, a-1), D(a, a), D(a, a+1)
        double2 dg, lo = cd(0.0, 0.0), up = cd(0.0, 0.0);
        Line1D k = line1d(a, a, ny, P.hy, wv);
        dg = cd(-P.c * k.s + k.w + ds.x * k.m, (2.0 / P.dt + ds.y) * k.m);
        if (a > 0) {
            Line1D kl = line1d(a, a - 1, ny, P.hy, wv);
            lo = cd(-P.c * kl.s + kl.w + ds.x * kl.m, (2.0 / P.dt + ds.y) * kl.m);
        }
        if (a < ny - 1) {
            Line1D ku = line1d(a, a + 1, ny, P.hy, wv);
            up = cd(-P.c * ku.s + ku.w + ds.x * ku.m, (2.0 / P.dt + ds.y) * ku.m);
        }
        const double2 den = csub(dg, cmul(lo, prev_cp));
        const double2 iv = cinv(den);
        const double2 c1 = cmul(up, iv);
        sub[o + a] = lo;
        inv[o + a] = iv;
        cp[o + a] = c1;
        prev_cp = c1;
    }
}

// (M^G x)_a on a line of ny nodes (x read through xv(b)).
template <class XF>
__device__ __forceinline__ double2 mass_apply1d(int a, int ny, double hy, XF xv) {
    double2 acc = cd(0.0, 0.0);
    for (int b = max(a - 1, 0); b <= min(a + 1, ny - 1); ++b) {
        double mm = 0.0;
        const int lo = max(max(a, b) - 1, 0), hi = min(min(a, b), ny - 2);
        for (int e = lo; e <= hi; ++e) mm += hy * ref_mass(a - e, b - e);
        acc = cadd(acc, cscale(mm, xv(b)));
    }
    return acc;
}

// G_e[:, j] = scale * sum_s a_s d_s D_{e,s}^{-1} M^G e_j: thread per (edge,
// column j); the forward sweep starts at row j - 1 (the right-hand side is
// zero above it); X holds the forward values of one edge (row-major, so the
// threads of a row store and load contiguously).
__global__ void pade_G_kernel(int ny, double hy, int e0, int ecount, int m, const double2 *ad,
                              const double2 *sub, const double2 *cp, const double2 *inv,
                              double2 *X, double2 *G, double2 scale) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int el = blockIdx.y;            // edge within this batch
    if (j >= ny || el >= ecount) return;
    const int e = e0 + el;
    const long nn = (long)ny * ny;
    double2 *Xe = X + (long)el * nn;
    double2 *Ge = G + (long)el * nn;
    auto rhs = [&](int a) -> double2 {
        if (a < j - 1 || a > j + 1) return cd(0.0, 0.0);
        double mm = 0.0;
        const int lo = max(max(a, j) - 1, 0), hi = min(min(a, j), ny - 2);
        for (int q = lo; q <= hi; ++q) mm += hy * ref_mass(a - q, j - q);
        return cd(mm, 0.0);
    };
    const int a0 = max(j - 1, 0);
    for (int s = 0; s < m; ++s) {
        const long o = ((long)e * m + s) * ny;
        const double2 w = cmul(cmul(ad[2 * s], ad[2 * s + 1]), scale);
        double2 y = cd(0.0, 0.0);
        for (int a = a0; a < ny; ++a) {
            y = cmul(csub(rhs(a), cmul(sub[o + a], y)), inv[o + a]);
            Xe[(long)a * ny + j] = y;
        }
        double2 x = cd(0.0, 0.0);
        for (int a = ny - 1; a >= 0; --a) {
            const double2 ya = a >= a0 ? Xe[(long)a * ny + j] : cd(0.0, 0.0);
            x = csub(ya, cmul(cp[o + a], x));
            const long g = (long)a * ny + j;
            Ge[g] = s == 0 ? cmul(w, x) : cadd(Ge[g], cmul(w, x));
        }
    }
}

// F[lines[b]] += -i c M^G G_{edges[b]} on the upper 64 x 64 tiles (the part
// of a Schur complement the factor's sweep reads).  G holds the batch's
// edges at G + (edges[b] - e0) * ny * ny.
template <typename T>
__global__ void pade_edge_add_kernel(int n, typename cplx_of<T>::type *F, const int *lines,
                                     const int *edges, int e0, const double2 *G, double c,
                                     double hy) {
    typedef typename cplx_of<T>::type T2;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y, b = blockIdx.z;
    if (col >= n || (r >> 6) > (col >> 6)) return;
    const int e = edges[b];
    if (e < 0) return;
    const double2 *Ge = G + (long)(e - e0) * n * n;
    const double2 mg = mass_apply1d(r, n, hy, [&](int k) { return Ge[(long)k * n + col]; });
    // -i c mg
    T2 *f = F + (long)lines[b] * n * n + (long)r * n + col;
    const T2 v = *f;
    T2 o;
    o.x = (T)((double)v.x + c * mg.y);
    o.y = (T)((double)v.y - c * mg.x);
    *f = o;
}

// Fixed-point residual of the edge functions and its eliminated right-hand
// side: thread per (edge, s), z_s = D_s^{-1}(M^G zeta_e - (D_s + M^G_f) phi_s).
__global__ void pade_phi_residual_kernel(Phys P, const StripMeta *strips, const double *W,
                                         int nedge, int m, const double2 *ad,
                                         const double2 *sub, const double2 *cp,
                                         const double2 *inv, const double2 *zeta,
                                         const double2 *phi, double2 *z, const StepCtl *c) {
    if (c && fp_idle(c)) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nedge * m) return;
    const int e = t / m, s = t % m, ny = P.ny;
    const double2 *ze = zeta + (long)edge_pline(strips, e) * ny;
    const double *Wl = W + (long)edge_gline(strips, e, nedge) * ny;
    const double2 ds = ad[2 * s + 1];
    const long o = (long)t * ny;
    const double2 *ph = phi + o;
    auto wv = [&](int k) -> double { return Wl[k]; };
    auto fv = [&](int k) -> double {
        const double2 q = ze[k];
        return P.beta * (q.x * q.x + q.y * q.y);
    };
    double2 y = cd(0.0, 0.0);
    for (int a = 0; a < ny; ++a) {
        double2 r = mass_apply1d(a, ny, P.hy, [&](int b) { return ze[b]; });
        for (int b = max(a - 1, 0); b <= min(a + 1, ny - 1); ++b) {
            const Line1D k = line1d(a, b, ny, P.hy, wv);
            const Line1D kf = line1d(a, b, ny, P.hy, fv);
            const double2 d = cd(-P.c * k.s + k.w + kf.w + ds.x * k.m, (2.0 / P.dt + ds.y) * k.m);
            r = csub(r, cmul(d, ph[b]));
        }
        y = cmul(csub(r, cmul(sub[o + a], y)), inv[o + a]);
        z[o + a] = y;
    }
    double2 x = cd(0.0, 0.0);
    for (int a = ny - 1; a >= 0; --a) {
        x = csub(z[o + a], cmul(cp[o + a], x));
        z[o + a] = x;
    }
}

// res(edge line) += i c M^G sum_s a_s d_s z_s: thread per (edge, node).
__global__ void pade_edge_rhs_kernel(Phys P, const StripMeta *strips, int nedge, int m,
                                     const double2 *ad, const double2 *z, double2 *res,
                                     const StepCtl *c) {
    if (c && fp_idle(c)) return;
    const int a = blockIdx.x * blockDim.x + threadIdx.x, e = blockIdx.y;
    const int ny = P.ny;
    if (a >= ny || e >= nedge) return;
    auto w = [&](int b) -> double2 {
        double2 acc = cd(0.0, 0.0);
        for (int s = 0; s < m; ++s)
            acc = cadd(acc, cmul(cmul(ad[2 * s], ad[2 * s + 1]), z[((long)e * m + s) * ny + b]));
        return acc;
    };
    const double2 mw = mass_apply1d(a, ny, P.hy, w);
    double2 *rr = res + (long)edge_pline(strips, e) * ny + a;
    const double2 v = *rr;
    *rr = cd(v.x - P.c * mw.y, v.y + P.c * mw.x);
}

// phi_s += z_s + D_s^{-1} M^G dzeta_e: thread per (edge, s).
__global__ void pade_phi_update_kernel(Phys P, const StripMeta *strips, int nedge, int m,
                                       const double2 *sub, const double2 *cp, const double2 *inv,
                                       const double2 *delta, const double2 *z, double2 *phi,
                                       double2 *work, const StepCtl *c) {
    if (c && fp_idle(c)) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nedge * m) return;
    const int e = t / m, ny = P.ny;
    const double2 *de = delta + (long)edge_pline(strips, e) * ny;
    const long o = (long)t * ny;
    double2 y = cd(0.0, 0.0);
    for (int a = 0; a < ny; ++a) {
        const double2 r = mass_apply1d(a, ny, P.hy, [&](int b) { return de[b]; });
        y = cmul(csub(r, cmul(sub[o + a], y)), inv[o + a]);
        work[o + a] = y;
    }
    double2 x = cd(0.0, 0.0);
    for (int a = ny - 1; a >= 0; --a) {
        x = csub(work[o + a], cmul(cp[o + a], x));
        phi[o + a] = cadd(phi[o + a], cadd(z[o + a], x));
    }
}

// psi_e = sum_s a_s d_s phi_{e,s}: thread per (edge, node).
__global__ void pade_psi_kernel(int ny, int nedge, int m, const double2 *ad, const double2 *phi,
                                double2 *psi, const StepCtl *c, int guard) {
    if (guard && c && fp_idle(c)) return;
    const int a = blockIdx.x * blockDim.x + threadIdx.x, e = blockIdx.y;
    if (a >= ny || e >= nedge) return;
    double2 acc = cd(0.0, 0.0);
    for (int s = 0; s < m; ++s)
        acc = cadd(acc, cmul(cmul(ad[2 * s], ad[2 * s + 1]), phi[((long)e * m + s) * ny + a]));
    psi[(long)e * ny + a] = acc;
}

// phi = 0, psi = 0 (start of a fixed point from u_{n-1}); guarded like the
// fixed point's other kernels when c is given (a Schwarz iteration that
// restarts its fixed points).
__global__ void pade_reset_kernel(long nphi, double2 *phi, long npsi, double2 *psi,
                                  const StepCtl *c) {
    if (c && (c->k_done || c->bad)) return;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nphi) phi[t] = cd(0.0, 0.0);
    if (t < npsi) psi[t] = cd(0.0, 0.0);
}

// out = -2i sa X (- I when add_eye): the local part of an L_h block with
// S_pade (S v = -i sa v + i G v), the G part added by a GEMM.
__global__ void pade_lh_form_kernel(int n, const double2 *X, double2 sa, int add_eye,
                                    double2 *out) {
    const int r = blockIdx.y, c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double2 x = X[(long)r * n + c];
    double2 o = cmul(cd(2.0 * sa.y, -2.0 * sa.x), x);
    if (add_eye && r == c) o.x -= 1.0;
    out[(long)r * n + c] = o;
}

inline unsigned blocks(long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_pade_lu(hipStream_t st, const Phys &P, const StripMeta *strips, const double *W,
                          int nedge, int with_free, int m, const double2 *ad, double2 *sub,
                          double2 *cp, double2 *inv, int e_first) {
    const int ne = nedge + (with_free ? 1 : 0);
    if (e_first >= ne) return hipSuccess;
    hipLaunchKernelGGL(pade_lu_kernel, dim3(blocks((long)(ne - e_first) * m, 64)), dim3(64), 0, st,
                       P, strips, W, nedge, with_free, e_first, m, ad, sub, cp, inv);
    return hipGetLastError();
}

hipError_t launch_pade_G(hipStream_t st, int ny, double hy, int e0, int ecount, int m,
                         const double2 *ad, const double2 *sub, const double2 *cp,
                         const double2 *inv, double2 *X, double2 *G, double2 scale) {
    if (ecount <= 0) return hipSuccess;
    hipLaunchKernelGGL(pade_G_kernel, dim3(blocks(ny, 64), ecount), dim3(64), 0, st, ny, hy, e0,
                       ecount, m, ad, sub, cp, inv, X, G, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pade_edge_add(hipStream_t st, int n, typename cplx_of<T>::type *F,
                                const int *lines, const int *edges, int batch, int e0,
                                const double2 *G, double c, double hy) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(pade_edge_add_kernel<T>, dim3(blocks(n, 256), n, batch), dim3(256), 0, st,
                       n, F, lines, edges, e0, G, c, hy);
    return hipGetLastError();
}
template hipError_t launch_pade_edge_add<double>(hipStream_t, int, double2 *, const int *,
                                                 const int *, int, int, const double2 *, double,
                                                 double);
template hipError_t launch_pade_edge_add<float>(hipStream_t, int, float2 *, const int *,
                                                const int *, int, int, const double2 *, double,
                                                double);

hipError_t launch_pade_fp_residual(hipStream_t st, const Phys &P, const StripMeta *strips,
                                   const double *W, int nedge, int m, const double2 *ad,
                                   const double2 *sub, const double2 *cp, const double2 *inv,
                                   const double2 *zeta, const double2 *phi, double2 *z,
                                   double2 *res, const StepCtl *c) {
    hipLaunchKernelGGL(pade_phi_residual_kernel, dim3(blocks((long)nedge * m, 64)), dim3(64), 0, st,
                       P, strips, W, nedge, m, ad, sub, cp, inv, zeta, phi, z, c);
    hipLaunchKernelGGL(pade_edge_rhs_kernel, dim3(blocks(P.ny, 256), nedge), dim3(256), 0, st, P,
                       strips, nedge, m, ad, z, res, c);
    return hipGetLastError();
}

hipError_t launch_pade_fp_update(hipStream_t st, const Phys &P, const StripMeta *strips, int nedge,
                                 int m, const double2 *ad, const double2 *sub, const double2 *cp,
                                 const double2 *inv, const double2 *delta, const double2 *z,
                                 double2 *phi, double2 *work, double2 *psi, const StepCtl *c) {
    hipLaunchKernelGGL(pade_phi_update_kernel, dim3(blocks((long)nedge * m, 64)), dim3(64), 0, st,
                       P, strips, nedge, m, sub, cp, inv, delta, z, phi, work, c);
    hipLaunchKernelGGL(pade_psi_kernel, dim3(blocks(P.ny, 256), nedge), dim3(256), 0, st, P.ny,
                       nedge, m, ad, phi, psi, c, 1);
    return hipGetLastError();
}

hipError_t launch_pade_reset(hipStream_t st, long nphi, double2 *phi, long npsi, double2 *psi,
                             const StepCtl *c) {
    const long n = nphi > npsi ? nphi : npsi;
    hipLaunchKernelGGL(pade_reset_kernel, dim3(blocks(n, 256)), dim3(256), 0, st, nphi, phi, npsi,
                       psi, c);
    return hipGetLastError();
}

hipError_t launch_pade_lh_form(hipStream_t st, int n, const double2 *X, double2 sa, int add_eye,
                               double2 *out) {
    hipLaunchKernelGGL(pade_lh_form_kernel, dim3(blocks(n, 256), n), dim3(256), 0, st, n, X, sa,
                       add_eye, out);
    return hipGetLastError();
}
