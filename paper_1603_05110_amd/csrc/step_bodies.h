// Per-node, per-line and per-instance bodies of the time-step kernels.  The
// single-instance kernels (kernels_assemble.hip, kernels_control.hip) and the
// batched kernels (kernels_batch.hip, which look the instance up in a table)
// call the same bodies, so both paths do the same arithmetic in the same
// order.  Device code only.
#pragma once

#include "osm_internal.h"

// Integrals between node (i,a) and node (ip,b) of one strip with nx lines:
// mass m, stiffness s, potential-weighted mass w = int phi_h psi psi (phi
// replaced by its Q1 interpolant, triple products exact) and the y-mass of
// the left/right edge lines (boundary mass M^Gamma).  Elements of the strip
// only: a strip is its own finite-element domain (Section 2.2).
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

// The fixed point of the current Schwarz map needs no more work.
__device__ __forceinline__ bool fp_idle(const StepCtl *c) {
    return c->q_conv || c->k_done || c->bad || c->q_fail;
}

// Fixed-point residual at strip node (L, a), residual form of the fixed
// point with the nonlinearity on the right-hand side:
//   res = 2i/dt M_j u_{j,n-1} - c M^Gamma Q^T (l_j; r_j) - K_j(W + beta|zeta|^2) zeta.
// With the factor of K_j(W), zeta + K_j(W)^{-1} res equals
// K_j(W)^{-1}(F - M_{beta|zeta|^2} zeta): the update of eq. localpbrobin.
//
// The Q1 integrals are summed element by element: the node's 3 x 3
// neighbourhood of zeta, u and phi = W + beta|zeta|^2 is loaded once, then
// each of the (up to) four elements around the node adds its entries with
// every corner (the same terms kparts() sums neighbour by neighbour).
__device__ __forceinline__ double2 residual_at(const Phys &P, const StripMeta *strips,
                                               const int *line_strip, const double *W,
                                               const double2 *u_old, const double2 *zeta,
                                               const double2 *g, int L, int a,
                                               const double2 *psi = nullptr) {
    const int ny = P.ny;
    const int j = line_strip[L];
    const StripMeta s = strips[j];
    const int i = L - s.off, nx = s.nx;
    const double *Wl = W + (long)s.line0 * ny;
    const double2 *ul = u_old + (long)s.line0 * ny;
    const double2 *zl = zeta + (long)s.off * ny;
    const double beta = P.beta, hx = P.hx, hy = P.hy, c = P.c, m2 = 2.0 / P.dt;
    const double2 *trace = nullptr;
    if (i == 0 && j >= 1) trace = g + (long)(2 * (j - 1) + 1) * ny;             // l_j
    if (i == nx - 1 && j <= P.nsub - 2) trace = g + (long)(2 * j) * ny;        // r_j
    // edge coefficient of M^Gamma on this line: i c (pe + i pe_im) M^Gamma
    // (Robin: p; S_pade^m: sum_s a_s), and with S_pade^m the edge functions'
    // term -sum_s B_s phi_s = i c M^Gamma psi (psi of this edge)
    const double pe = (i == 0 ? s.pl : 0.0) + (i == nx - 1 ? s.pr : 0.0);
    const double pe_im = (i == 0 ? s.pl_im : 0.0) + (i == nx - 1 ? s.pr_im : 0.0);
    const bool edge = i == 0 || i == nx - 1;
    const double2 *pse = (psi && edge) ? psi + (long)(2 * j + (i == 0 ? 0 : 1)) * ny : nullptr;
    double2 z[3][3], u[3][3], tr[3], ps[3];
    double ph[3][3];
#pragma unroll
    for (int di = 0; di < 3; ++di)
#pragma unroll
        for (int db = 0; db < 3; ++db) {
            const int ip = i + di - 1, b = a + db - 1;
            const bool ok = ip >= 0 && ip < nx && b >= 0 && b < ny;
            const long o = (long)ip * ny + b;
            z[di][db] = ok ? zl[o] : cd(0.0, 0.0);
            u[di][db] = ok ? ul[o] : cd(0.0, 0.0);
            const double wv = ok ? Wl[o] : 0.0;
            ph[di][db] = wv + beta * (z[di][db].x * z[di][db].x + z[di][db].y * z[di][db].y);
        }
#pragma unroll
    for (int db = 0; db < 3; ++db) {
        const int b = a + db - 1;
        tr[db] = (trace && b >= 0 && b < ny) ? trace[b] : cd(0.0, 0.0);
        ps[db] = (pse && b >= 0 && b < ny) ? pse[b] : cd(0.0, 0.0);
    }
    double2 acc = cd(0.0, 0.0);
#pragma unroll
    for (int exo = -1; exo <= 0; ++exo) {
        const int ex = i + exo;
        if (ex < 0 || ex > nx - 2) continue;
        const int Ax = -exo;
#pragma unroll
        for (int eyo = -1; eyo <= 0; ++eyo) {
            const int ey = a + eyo;
            if (ey < 0 || ey > ny - 2) continue;
            const int Ay = -eyo;
#pragma unroll
            for (int Bx = 0; Bx < 2; ++Bx)
#pragma unroll
                for (int By = 0; By < 2; ++By) {
                    const int di = exo + Bx + 1, db = eyo + By + 1;   // corner in the 3 x 3 block
                    const double mx = hx * ref_mass(Ax, Bx), sx = ref_stiff(Ax, Bx) / hx;
                    const double my = hy * ref_mass(Ay, By), sy = ref_stiff(Ay, By) / hy;
                    const double m = mx * my, st = sx * my + mx * sy;
                    double w = 0.0;
#pragma unroll
                    for (int cx = 0; cx < 2; ++cx)
#pragma unroll
                        for (int cy = 0; cy < 2; ++cy)
                            w += ph[exo + cx + 1][eyo + cy + 1] * ref_triple(cx, Ax, Bx) *
                                 ref_triple(cy, Ay, By);
                    w *= hx * hy;
                    const double2 zb = z[di][db], ub = u[di][db];
                    // 2i/dt m (u - z)
                    const double2 du = csub(ub, zb);
                    acc.x += -m2 * m * du.y;
                    acc.y += m2 * m * du.x;
                    // + c s z - w z
                    const double cs = c * st - w;
                    acc.x += cs * zb.x;
                    acc.y += cs * zb.y;
                    if (edge && Bx == Ax) {
                        // - i c (pe + i pe_im) M^Gamma z - c M^Gamma trace
                        // + i c M^Gamma psi (same line only)
                        const double e = c * pe * my, ei = c * pe_im * my, cm = c * my;
                        acc.x += e * zb.y + ei * zb.x;
                        acc.y += -e * zb.x + ei * zb.y;
                        acc.x -= cm * tr[db].x;
                        acc.y -= cm * tr[db].y;
                        acc.x -= cm * ps[db].y;
                        acc.y += cm * ps[db].x;
                    }
                }
        }
    }
    return acc;
}

// zeta <- u_{n-1} restricted to the strips (interface lines copied).
__device__ __forceinline__ void copy_u_at(const Phys &P, const StripMeta *strips,
                                          const int *line_strip, const double2 *u,
                                          double2 *zeta, int L, int a) {
    StripMeta s = strips[line_strip[L]];
    int gl = s.line0 + (L - s.off);
    zeta[(long)L * P.ny + a] = u[(long)gl * P.ny + a];
}

// zeta += delta on packed line L; per-line partial sums |delta|^2, |zeta|^2
// and a non-finite counter.  Block of 256 threads.
__device__ __forceinline__ void update_norms_line(int ny, double2 *zeta, const double2 *delta,
                                                  double *part, int L) {
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

// Flux update of trace t, eq. fluxlr with S = -ip (Jacobi):
//   new r_i     = -l_{i+1} - 2ip v_{i+1}(first line)
//   new l_{i+1} = -r_i     - 2ip v_i(last line)
// Per-trace partial sums of |gn - g|^2 and |gn|^2.  Block of 256 threads.
__device__ __forceinline__ void flux_trace(const Phys &P, const StripMeta *strips,
                                           const double2 *g, const double2 *v, double2 *gn,
                                           double *part, int t, const double2 *psi = nullptr) {
    int ny = P.ny;
    int i = t >> 1;
    const double2 *src;
    const double2 *vt;
    const double2 *pe = nullptr;
    if ((t & 1) == 0) {           // r_i from strip i+1's left line
        src = g + (long)(2 * i + 1) * ny;
        vt = v + (long)strips[i + 1].off * ny;
        if (psi) pe = psi + (long)(2 * (i + 1)) * ny;
    } else {                      // l_{i+1} from strip i's right line
        src = g + (long)(2 * i) * ny;
        StripMeta s = strips[i];
        vt = v + (long)(s.off + s.nx - 1) * ny;
        if (psi) pe = psi + (long)(2 * i + 1) * ny;
    }
    // new trace = -x + 2 S w with S w = -i t w + i psi, t = P.tre + i P.tim
    // (Robin: t = p, psi = 0)
    const double tr2 = 2.0 * P.tre, ti2 = 2.0 * P.tim;
    double sd = 0.0, sn = 0.0;
    for (int a = threadIdx.x; a < ny; a += blockDim.x) {
        double2 x = src[a], w = vt[a];
        double2 r = cd(-x.x + tr2 * w.y + ti2 * w.x, -x.y - tr2 * w.x + ti2 * w.y);
        if (pe) {
            const double2 q = pe[a];
            r.x -= 2.0 * q.y;
            r.y += 2.0 * q.x;
        }
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

// u_n = 2 vbar - u_{n-1} at global node (gl, a); vbar is the strip value,
// the mean of the two copies on an interface line.
__device__ __forceinline__ void time_update_at(const Phys &P, const int2 *gmap, const double2 *v,
                                               double2 *u, int gl, int a) {
    int ny = P.ny;
    int2 m = gmap[gl];
    double2 vb = v[(long)m.x * ny + a];
    if (m.y >= 0) vb = cscale(0.5, cadd(vb, v[(long)m.y * ny + a]));
    long o = (long)gl * ny + a;
    double2 uo = u[o];
    u[o] = cd(2.0 * vb.x - uo.x, 2.0 * vb.y - uo.y);
}

// Partial of u* M u over global line gl with the global Q1 mass
// M = M1x (x) M1y.  Block of 256 threads.
__device__ __forceinline__ void mass_line(const Phys &P, const double2 *u, double *part, int gl) {
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

// Deterministic sum of n strided values into out[0 .. stride).  One block of
// 256 threads.
__device__ __forceinline__ void sum_block(const double *part, int n, int stride, double *out) {
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

__device__ __forceinline__ double ctl_wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double ctl_block_sum(double v, double *red) {
    v = ctl_wsum(v);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// Thread 0 only.
__device__ __forceinline__ void step_init_body(StepCtl *c, const StepCfg &cfg) {
    c->cfg = cfg;
    c->q_conv = 0; c->q_iter = 0; c->q_total = 0; c->q_fail = 0;
    c->r_done = 0; c->k = 0; c->k_done = 0; c->bad = 0; c->commit = 0;
    c->gm_total = 0;
    c->ready = 1;
    c->tq = cfg.tol_q;
    c->inc = 0.0; c->ref = 0.0;
    // the first inner tolerance of this step follows the first increment of
    // the last one (how far the start of the iteration was from its map)
    c->prev_rel = c->first_rel > 0.0 ? fmin(1.0, c->first_rel) : 1.0;
    c->rho = 0.0;
}

// Start of a Schwarz iteration (thread 0 only): new fixed point, tolerance
// from the previous increment (inexact inner solves), GMRES cycle idle.
__device__ __forceinline__ void iter_reset_body(StepCtl *c, GmresCtl *g) {
    c->q_conv = 0;
    c->q_iter = 0;
    c->q_fail = 0;
    c->r_done = 0;
    c->commit = 0;
    c->ready = 0;
    double t = c->cfg.tol_q;
    if (c->cfg.eta_q > 0.0) t = fmax(t, c->cfg.eta_q * fmin(1.0, c->prev_rel));
    c->tq = t;
    if (g) { g->done = 1; g->finished = 0; g->conv = 0; g->j = 0; g->total = 0; }
}

// Fixed-point test of every strip from the per-line partial sums:
// converged when ||dzeta_j|| <= tq ||zeta_j|| for all strips j (or after
// fixed_q iterations).  With the error-estimate test (cfg.q_est, dprev
// given) the factor r/(1-r) multiplies ||dzeta_j|| from the step's second
// Schwarz iteration on: for a map with contraction factor r, the distance
// of zeta^q to the fixed point is at most r/(1-r) ||zeta^q - zeta^{q-1}||.
// r is twice the largest ratio ||dzeta^2|| / ||dzeta^1|| over the strips
// measured in the step (dprev keeps each strip's last ||dzeta||^2); the
// test is used only while r < 1/2.  One block.
__device__ __forceinline__ void q_check_block(const Phys &P, const StripMeta *strips,
                                              const double *part, StepCtl *c,
                                              double *dprev = nullptr) {
    __shared__ int notconv, nonfinite;
    __shared__ unsigned long long rho_bits;
    if (threadIdx.x == 0) { notconv = 0; nonfinite = 0; rho_bits = 0ull; }
    __syncthreads();
    const double tq = c->tq;
    const double r = 2.0 * c->rho;
    const bool est = dprev && c->cfg.q_est && c->k >= 1 && r > 0.0 && r < 0.5;
    const double fac = est ? r / (1.0 - r) : 1.0;
    const bool measure = dprev && c->q_iter >= 1;   // second or later iterate
    // one wave per strip, its lanes over the strip's lines (all loads of a
    // strip in flight together), summed by the fixed butterfly of ctl_wsum
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int j = wave; j < P.nsub; j += nw) {
        const StripMeta s = strips[j];
        double d = 0, z = 0, b = 0;
        for (int i = lane; i < s.nx; i += 64) {
            d += part[3 * (s.off + i)];
            z += part[3 * (s.off + i) + 1];
            b += part[3 * (s.off + i) + 2];
        }
        d = ctl_wsum(d);
        z = ctl_wsum(z);
        b = ctl_wsum(b);
        if (lane == 0) {
            if (b > 0 || !isfinite(d) || !isfinite(z)) atomicOr(&nonfinite, 1);
            if (!(fac * sqrt(d) <= tq * sqrt(z))) atomicOr(&notconv, 1);
            if (dprev) {
                if (measure && dprev[j] > 0.0 && isfinite(d)) {
                    // non-negative doubles order like their bit patterns
                    const double ratio = sqrt(d / dprev[j]);
                    atomicMax(&rho_bits, (unsigned long long)__double_as_longlong(ratio));
                }
                dprev[j] = d;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (measure && c->q_iter == 1) c->rho = fmax(c->rho, __longlong_as_double((long long)rho_bits));
    c->q_iter += 1;
    c->q_total += 1;
    if (nonfinite) { c->bad = 1; return; }
    bool conv = c->cfg.fixed_q > 0 ? (c->q_iter >= c->cfg.fixed_q) : !notconv;
    if (conv) c->q_conv = 1;
    else if (c->q_iter >= c->cfg.max_q) c->q_fail = 1;
}

// End of the Schwarz map: ||g^{k+1} - g^k||, ||g^{k+1}|| from the flux
// partials.  Classical algorithm: decide convergence and commit g <- R(g).
// One block.
__device__ __forceinline__ void flux_finalize_block(const double *part, int nt, StepCtl *c) {
    __shared__ double red[16];
    double a = 0, b = 0;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) { a += part[2 * t]; b += part[2 * t + 1]; }
    a = ctl_block_sum(a, red);
    b = ctl_block_sum(b, red);
    if (threadIdx.x != 0) return;
    c->r_done = 1;
    if (!c->cfg.classical) return;
    double inc = sqrt(a), ref = sqrt(b);
    if (!isfinite(inc)) { c->bad = 1; return; }
    c->commit = 1;
    c->ready = 1;
    c->k += 1;
    c->inc = inc;
    c->ref = ref;
    c->prev_rel = inc / fmax(ref, 1e-300);
    if (c->k == 1) c->first_rel = c->prev_rel;
    double thr = c->cfg.tol_k_rel ? c->cfg.tol_k * fmax(ref, 1e-300) : c->cfg.tol_k;
    if (c->cfg.fixed_k > 0) { if (c->k >= c->cfg.fixed_k) c->k_done = 1; }
    else if (inc < thr) c->k_done = 1;
}
