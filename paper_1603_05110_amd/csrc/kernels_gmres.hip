// Interface-space kernels of the preconditioned algorithm (Section 3,
// eq. Lmpi; Section 4.2): the block matrix-vector product with L_h and the
// vector primitives of GMRES on P x = y, P = I - L_h.  FP64.
#include "osm_internal.h"

#include <algorithm>

namespace {

__device__ __forceinline__ double wsum(double v) { return wave_sum_f64(v); }

// Row a of output trace t of L_h x (eq. Lmpi): trace 2i (new r_i) is fed by
// strip i+1 through X^{i+1,1} l_{i+1} + X^{i+1,2} r_{i+1}; trace 2i+1 (new
// l_{i+1}) by strip i through X^{i,3} l_i + X^{i,4} r_i.  LH holds, per
// block set, the four dense blocks X^{.,1..4} (row-major ny x ny).
// mode_p = 1: y = x - L_h x (the preconditioner P), else y = L_h x.
__device__ __forceinline__ void lh_matvec_body(Phys P, const StripMeta *strips,
                                               const double2 *LH, const double2 *x, double2 *y,
                                               int mode_p);

// Workgroup b -> (trace, tile of 4 rows).  Workgroups are dispatched to the 8
// XCDs round-robin; all traces of one row tile are given to consecutive
// workgroups of one XCD, so the tile's rows of the (shared) blocks X^{.,1..4}
// are read from HBM once and then from that XCD's L2.
__device__ __forceinline__ bool lh_tile_of(int b, int ntr, int ntile, int *t, int *tile) {
    int xcd = b & 7, m = b >> 3;
    *t = m % ntr;
    *tile = (m / ntr) * 8 + xcd;
    return *tile < ntile;
}

__global__ __launch_bounds__(256) void lh_matvec_kernel(Phys P, const StripMeta *strips,
                                                        const double2 *LH, const double2 *x,
                                                        double2 *y, int mode_p) {
    lh_matvec_body(P, strips, LH, x, y, mode_p);
}

__device__ __forceinline__ void lh_matvec_body(Phys P, const StripMeta *strips,
                                               const double2 *LH, const double2 *x, double2 *y,
                                               int mode_p) {
    int n = P.ny;
    int t, tile;
    if (!lh_tile_of(blockIdx.x, 2 * (P.nsub - 1), (n + 3) / 4, &t, &tile)) return;
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int a = tile * 4 + wave;
    if (a >= n) return;
    int i = t >> 1;
    int strip, blk_l, blk_r, src_l, src_r;
    if ((t & 1) == 0) {          // from strip i+1: inputs l_{i+1} (trace 2i+1), r_{i+1} (trace 2i+2)
        strip = i + 1; blk_l = 0; blk_r = 1;
        src_l = 2 * i + 1;
        src_r = (i + 1 <= P.nsub - 2) ? 2 * (i + 1) : -1;
    } else {                     // from strip i: inputs l_i (trace 2i-1), r_i (trace 2i)
        strip = i; blk_l = 2; blk_r = 3;
        src_l = (i >= 1) ? 2 * (i - 1) + 1 : -1;
        src_r = 2 * i;
    }
    long nn = (long)n * n;
    const double2 *base = LH + (long)strips[strip].cls * 4 * nn;
    double sr = 0.0, si = 0.0;
    if (src_l >= 0) {
        const double2 *row = base + blk_l * nn + (long)a * n;
        const double2 *v = x + (long)src_l * n;
        for (int c = lane; c < n; c += 64) {
            double2 m = row[c], w = v[c];
            sr += m.x * w.x - m.y * w.y;
            si += m.x * w.y + m.y * w.x;
        }
    }
    if (src_r >= 0) {
        const double2 *row = base + blk_r * nn + (long)a * n;
        const double2 *v = x + (long)src_r * n;
        for (int c = lane; c < n; c += 64) {
            double2 m = row[c], w = v[c];
            sr += m.x * w.x - m.y * w.y;
            si += m.x * w.y + m.y * w.x;
        }
    }
    sr = wsum(sr);
    si = wsum(si);
    if (lane == 0) {
        long o = (long)t * n + a;
        if (mode_p) {
            double2 xv = x[o];
            y[o] = cd(xv.x - sr, xv.y - si);
        } else {
            y[o] = cd(sr, si);
        }
    }
}

// L_h x with every block row reused over many strips.  Workgroup
// (class, group, tile) of the plan owns rows [a0, a0 + 2R) of the blocks of
// one strip class.  Wave w computes output side w & 1 for R rows: side 0 is
// trace 2(j-1) (new r_{j-1}) = X^1 l_j + X^2 r_j, side 1 is trace 2j+1
// (new l_{j+1}) = X^3 l_j + X^4 r_j (eq. Lmpi; l_0 and r_{N-1} are zero).
// It keeps its R rows of its two blocks in registers and loops over its
// group's strips of that class, writing each result itself; every output
// trace has exactly one writer.  The inputs l_j, r_j of SB strips at a time
// are loaded together and staged in LDS, so one memory latency serves SB
// strips.
//
// DOTS (Arnoldi step, y = x - L_h x with x = V_{nv-1}): the kernel also
// forms the first Gram-Schmidt pass's partial products V_k^H y over the
// outputs it wrote, k < nv <= 64: lane k loads V_k at each output (lane
// nv-1 thereby holds x), accumulates conj(V_k) y, and the workgroup writes
// its nv partials to part[block][k] (stride ld), summed in a fixed order.
template <int NCH, int R, int SB, bool DOTS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void lh_matvec_reg_kernel(
    Phys P, const LhClass *ctab, int ncls, const int *clist, int tiles, const double2 *LH,
    const double2 *x, double2 *y, int mode_p, const GmresCtl *ctl, const double2 *V, long ng,
    int nv, double2 *part, int ld) {
    if (ctl && ctl->done) return;
    constexpr int W = NCH * 64, SPT = (2 * W + 255) / 256;
    __shared__ double2 stage[SB][2 * W];   // [strip of the batch][l_j | r_j]
    const int n = P.ny, N = P.nsub;
    int pc = 0;
    while (pc + 1 < ncls && (int)blockIdx.x >= ctab[pc + 1].block_off) ++pc;
    const LhClass C = ctab[pc];
    const int cls = C.cls, G = C.groups, loc = (int)blockIdx.x - C.block_off;
    const int tile = loc % tiles, group = loc / tiles;
    const int ns = (C.count - group + G - 1) / G;   // this group's strips (ranks group + G i)
    const int *mine = clist + C.list_off + group;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int side = wave & 1, r0 = tile * 2 * R + (wave >> 1) * R;
    const long nn = (long)n * n;
    const double2 *B0 = LH + ((long)cls * 4 + 2 * side) * nn;   // multiplies l_j
    const double2 *B1 = B0 + nn;                                // multiplies r_j
    double2 m0[R][NCH], m1[R][NCH];
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            int row = r0 + rr, col = c * 64 + lane;
            bool ok = row < n && col < n;
            m0[rr][c] = ok ? B0[(long)row * n + col] : cd(0.0, 0.0);
            m1[rr][c] = ok ? B1[(long)row * n + col] : cd(0.0, 0.0);
        }
    auto has_out = [&](int j) { return side == 0 ? j >= 1 : j <= N - 2; };
    auto out_trace = [&](int j) { return side == 0 ? 2 * (j - 1) : 2 * j + 1; };
    double2 acc = cd(0.0, 0.0);
    for (int i0 = 0; i0 < ns; i0 += SB) {
        int js[SB];
#pragma unroll
        for (int b = 0; b < SB; ++b) js[b] = i0 + b < ns ? mine[G * (i0 + b)] : N;
        // every load of the batch in flight together
        double2 stg[SB][SPT];
#pragma unroll
        for (int b = 0; b < SB; ++b)
#pragma unroll
            for (int q = 0; q < SPT; ++q) {
                const int e = threadIdx.x + 256 * q, v = e >= W, col = e - v * W, j = js[b];
                const double2 *src =
                    j >= N ? nullptr
                           : (v == 0 ? (j >= 1 ? x + (long)(2 * (j - 1) + 1) * n : nullptr)
                                     : (j <= N - 2 ? x + (long)(2 * j) * n : nullptr));
                stg[b][q] = (e < 2 * W && src && col < n) ? src[col] : cd(0.0, 0.0);
            }
        double2 vk[SB][R];
        if constexpr (DOTS) {
#pragma unroll
            for (int b = 0; b < SB; ++b)
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int j = js[b], a = r0 + rr;
                    const bool ok = j < N && has_out(j) && lane < nv && a < n;
                    vk[b][rr] = ok ? V[(long)lane * ng + (long)out_trace(j) * n + a]
                                   : cd(0.0, 0.0);
                }
        }
        __syncthreads();   // the previous batch is no longer read
#pragma unroll
        for (int b = 0; b < SB; ++b)
#pragma unroll
            for (int q = 0; q < SPT; ++q) {
                const int e = threadIdx.x + 256 * q;
                if (e < 2 * W) stage[b][e] = stg[b][q];
            }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < SB; ++b) {
            const int j = js[b];
            if (j >= N || !has_out(j)) continue;
            const int t = out_trace(j);
            const double2 *sl = stage[b], *sr_ = stage[b] + W;
            double ar[R], ai[R];
#pragma unroll
            for (int rr = 0; rr < R; ++rr) { ar[rr] = 0.0; ai[rr] = 0.0; }
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const double2 wl = sl[c * 64 + lane], wr = sr_[c * 64 + lane];
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    ar[rr] += m0[rr][c].x * wl.x - m0[rr][c].y * wl.y + m1[rr][c].x * wr.x - m1[rr][c].y * wr.y;
                    ai[rr] += m0[rr][c].x * wl.y + m0[rr][c].y * wl.x + m1[rr][c].x * wr.y + m1[rr][c].y * wr.x;
                }
            }
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                double sr = wsum(ar[rr]), si = wsum(ai[rr]);
                int a = r0 + rr;
                if (a >= n) continue;
                long o = (long)t * n + a;
                if constexpr (DOTS) {
                    const double2 v = vk[b][rr];
                    const double xr = __shfl(v.x, nv - 1, 64), xi = __shfl(v.y, nv - 1, 64);
                    const double2 wo = cd(xr - sr, xi - si);
                    if (lane == 0) y[o] = wo;
                    acc.x += v.x * wo.x + v.y * wo.y;   // conj(V_k) y
                    acc.y += v.x * wo.y - v.y * wo.x;
                } else if (lane == 0) {
                    if (mode_p) {
                        double2 xv = x[o];
                        y[o] = cd(xv.x - sr, xv.y - si);
                    } else {
                        y[o] = cd(sr, si);
                    }
                }
            }
        }
    }
    if constexpr (DOTS) {
        __shared__ double2 red[4][64];
        red[wave][lane] = acc;
        __syncthreads();
        if (threadIdx.x < nv) {
            const int k = threadIdx.x;
            const long b = blockIdx.x;
            part[b * ld + k] = cadd(cadd(red[0][k], red[1][k]), cadd(red[2][k], red[3][k]));
        }
    }
}

// part[b * nv + k] = partial of V_k^H w over block b's slice.
__global__ __launch_bounds__(256) void multidot_kernel(long n, const double2 *V, int nv,
                                                       const double2 *w, double2 *part) {
    __shared__ double red_r[4], red_i[4];
    int nblk = gridDim.x;
    long chunk = (n + nblk - 1) / nblk;
    long lo = (long)blockIdx.x * chunk, hi = min(n, lo + chunk);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = 0; k < nv; ++k) {
        const double2 *vk = V + (long)k * n;
        double sr = 0.0, si = 0.0;
        for (long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
            double2 a = vk[e], b = w[e];
            sr += a.x * b.x + a.y * b.y;       // conj(a) * b
            si += a.x * b.y - a.y * b.x;
        }
        sr = wsum(sr);
        si = wsum(si);
        if (lane == 0) { red_r[wave] = sr; red_i[wave] = si; }
        __syncthreads();
        if (threadIdx.x == 0) {
            part[(long)blockIdx.x * nv + k] = cd(red_r[0] + red_r[1] + red_r[2] + red_r[3],
                                                 red_i[0] + red_i[1] + red_i[2] + red_i[3]);
        }
        __syncthreads();
    }
}

__global__ void multidot_finalize_kernel(const double2 *part, int nv, int nblk, double2 *out) {
    int k = threadIdx.x;
    if (k >= nv) return;
    double2 acc = cd(0.0, 0.0);
    for (int b = 0; b < nblk; ++b) acc = cadd(acc, part[(long)b * nv + k]);
    out[k] = acc;
}

// w -= sum_k h_k V_k  (sub = 1)  or  w += sum_k h_k V_k  (sub = 0)
__global__ void multiaxpy_kernel(long n, const double2 *V, int nv, const double2 *h,
                                 double2 *w, int sub) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double2 acc = cd(0.0, 0.0);
    for (int k = 0; k < nv; ++k) acc = cadd(acc, cmul(h[k], V[(long)k * n + e]));
    double2 o = w[e];
    w[e] = sub ? csub(o, acc) : cadd(o, acc);
}

__global__ __launch_bounds__(256) void norm_partials_kernel(long n, const double2 *x,
                                                            double *part) {
    __shared__ double red[4];
    int nblk = gridDim.x;
    long chunk = (n + nblk - 1) / nblk;
    long lo = (long)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double s = 0.0;
    for (long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double2 a = x[e];
        s += a.x * a.x + a.y * a.y;
    }
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void scale_copy_kernel(long n, const double2 *x, double2 s, double2 *y) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = cmul(s, x[e]);
}

__global__ void axpby_kernel(long n, double2 a, const double2 *x, double2 b, const double2 *y,
                             double2 *z) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) z[e] = cadd(cmul(a, x[e]), cmul(b, y[e]));
}

// ---------------------------------------------------------------------------
// GMRES with the Arnoldi loop driven on the device: every kernel below reads
// ctl->done first and returns at once when the cycle has converged, so the
// host can enqueue several iterations ahead and synchronise once per chunk.

// Classical Gram-Schmidt, twice, split over at most 256 contiguous chunks:
// each workgroup owns one chunk of w and writes its partial dot products
// with every basis vector; the next kernel reduces the partials of all
// chunks in a fixed order (deterministic).  part layout: [chunk][k], stride
// ld = m + 1.

__device__ __forceinline__ void chunk_range(long n, long *lo, long *hi) {
    long c = (n + gridDim.x - 1) / gridDim.x;
    *lo = min(n, (long)blockIdx.x * c);
    *hi = min(n, *lo + c);
}

// Partial of V_k^H w over this workgroup's chunk, for k < nv, into part.
__device__ __forceinline__ void chunk_dots(long n, const double2 *V, int nv, const double2 *w,
                                           long lo, long hi, double2 *part, int ld) {
    __shared__ double rr[4][64], ri[4][64];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k0 = 0; k0 < nv; k0 += 64) {
        int kn = min(64, nv - k0);
        for (int kk = 0; kk < kn; ++kk) {
            const double2 *vk = V + (long)(k0 + kk) * n;
            double sr = 0.0, si = 0.0;
            for (long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
                double2 a = vk[e], wv = w[e];
                sr += a.x * wv.x + a.y * wv.y;       // conj(a) * w
                si += a.x * wv.y - a.y * wv.x;
            }
            sr = wsum(sr);
            si = wsum(si);
            if (lane == 0) { rr[wave][kk] = sr; ri[wave][kk] = si; }
        }
        __syncthreads();
        if (threadIdx.x < kn) {
            int kk = threadIdx.x;
            part[(long)blockIdx.x * ld + k0 + kk] =
                cd(rr[0][kk] + rr[1][kk] + rr[2][kk] + rr[3][kk],
                   ri[0][kk] + ri[1][kk] + ri[2][kk] + ri[3][kk]);
        }
        __syncthreads();
    }
}

// dots[k] = sum over chunks of part[.][k], k < nv, into LDS (dots may be
// added to an existing value with add = 1).  A block of 256 threads splits
// every sum four ways (chunk b goes to quarter b % 4, four independent
// accumulators each) and adds the quarters in a fixed order, so the result
// is deterministic and the loads are in flight together.
__device__ __forceinline__ void reduce_dots(const double2 *part, int nb, int ld, int nv,
                                            double2 *dots, int add = 0) {
    __shared__ double2 q4[4][64];
    const int kk = threadIdx.x & 63, q = threadIdx.x >> 6;
    for (int k0 = 0; k0 < nv; k0 += 64) {
        int k = k0 + kk;
        double2 a0 = cd(0.0, 0.0), a1 = a0, a2 = a0, a3 = a0;
        if (k < nv) {
            int b = q;
            for (; b + 12 < nb; b += 16) {
                a0 = cadd(a0, part[(long)b * ld + k]);
                a1 = cadd(a1, part[(long)(b + 4) * ld + k]);
                a2 = cadd(a2, part[(long)(b + 8) * ld + k]);
                a3 = cadd(a3, part[(long)(b + 12) * ld + k]);
            }
            for (; b < nb; b += 4) a0 = cadd(a0, part[(long)b * ld + k]);
        }
        q4[q][kk] = cadd(cadd(a0, a1), cadd(a2, a3));
        __syncthreads();
        if (q == 0 && k < nv) {
            double2 t = cadd(cadd(q4[0][kk], q4[1][kk]), cadd(q4[2][kk], q4[3][kk]));
            dots[k] = add ? cadd(dots[k], t) : t;
        }
        __syncthreads();
    }
}

// dots[k] = sum over b < np of part[b * ld + k], k < nv <= 64, with all
// 256 threads: thread t sums the partials b = t / nv (mod S), S = 256 / nv,
// of k = t % nv, then the S slot sums are added in slot order (the result
// depends only on np and nv, so it is the same in every workgroup).
__device__ __forceinline__ void reduce_parts_wide(const double2 *part, int np, int ld, int nv,
                                                  double2 *dots) {
    __shared__ double2 slot_sum[256];
    const int S = 256 / nv, t = threadIdx.x;
    if (t < S * nv) {
        const int k = t % nv, sl = t / nv;
        double2 a0 = cd(0.0, 0.0), a1 = a0;
        int b = sl;
        for (; b + S < np; b += 2 * S) {
            a0 = cadd(a0, part[(long)b * ld + k]);
            a1 = cadd(a1, part[(long)(b + S) * ld + k]);
        }
        if (b < np) a0 = cadd(a0, part[(long)b * ld + k]);
        slot_sum[t] = cadd(a0, a1);
    }
    __syncthreads();
    if (t < nv) {
        double2 s = cd(0.0, 0.0);
        for (int sl = 0; sl < S; ++sl) s = cadd(s, slot_sum[sl * nv + t]);
        dots[t] = s;
    }
    __syncthreads();
}

// First pass: partial dots of w = V_{j+1} (the new Arnoldi vector) with V_0..V_j.
__global__ __launch_bounds__(256) void cgs_dots_kernel(long n, const double2 *V, int nv,
                                                       const double2 *w, double2 *part, int ld,
                                                       const GmresCtl *ctl) {
    if (ctl->done) return;
    long lo, hi;
    chunk_range(n, &lo, &hi);
    chunk_dots(n, V, nv, w, lo, hi, part, ld);
}

// w -= sum_k dots[k] V_k with the dots reduced from the nb partials of
// part_in; then either the partial dots of the updated w (second pass,
// part_out) or the chunk's partial of |w|^2 (norm_part).
__global__ __launch_bounds__(256) void cgs_update_kernel(long n, const double2 *V, int nv,
                                                         const double2 *part_in, int nb, int ld,
                                                         double2 *w, double2 *part_out,
                                                         double *norm_part, const GmresCtl *ctl) {
    if (ctl->done) return;
    __shared__ double2 dots[256];
    __shared__ double red[4];
    reduce_dots(part_in, nb, ld, nv, dots);
    long lo, hi;
    chunk_range(n, &lo, &hi);
    double s = 0.0;
    for (long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double2 acc = cd(0.0, 0.0);
        for (int k = 0; k < nv; ++k) acc = cadd(acc, cmul(dots[k], V[(long)k * n + e]));
        double2 o = csub(w[e], acc);
        w[e] = o;
        s += o.x * o.x + o.y * o.y;
    }
    if (part_out) {
        __syncthreads();   // this chunk of w is final (each element is read back by its writer)
        chunk_dots(n, V, nv, w, lo, hi, part_out, ld);
    } else {
        s = wsum(s);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) norm_part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

__device__ __forceinline__ double wave_reduce_parts(const double *part, int np) {
    int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int b = lane; b < np; b += 64) s += part[b];
    return wsum(s);
}

// Start of a cycle: beta = ||r|| from np partials, e = beta e_1, done when
// beta is already below tol * ||y|| (first cycle: ||y|| = beta).  One wave.
__global__ void gmres_begin_kernel(const double *part, int np, int first, double accept,
                                   double2 *e, int m, GmresCtl *ctl, const StepCtl *sc) {
    if (sc && (sc->r_done != 1 || sc->k_done || sc->bad)) return;
    double beta = sqrt(wave_reduce_parts(part, np));
    if (threadIdx.x != 0) return;
    ctl->finished = 0;
    if (first) ctl->total = 0;
    if (first) ctl->bnorm = beta;
    ctl->beta = beta;
    ctl->j = 0;
    ctl->done = 0;
    ctl->conv = 0;
    ctl->resid = beta;
    if (!isfinite(beta)) { ctl->bad = 1; ctl->done = 1; return; }
    if (beta <= accept * ctl->tol * ctl->bnorm || beta == 0.0) { ctl->done = 1; ctl->conv = 1; }
    ctl->inv_hn = beta > 0 ? 1.0 / beta : 0.0;
    for (int i = 0; i <= m; ++i) e[i] = cd(0.0, 0.0);
    e[0] = cd(beta, 0.0);
}

// y = s x with s = ctl->inv_hn (normalisation of the new Arnoldi vector)
__global__ void scale_ctl_kernel(long n, const double2 *x, double2 *y, const GmresCtl *ctl) {
    if (ctl->done && ctl->j > 0) return;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = cscale(ctl->inv_hn, x[e]);
}

// Column j of the Hessenberg matrix (h[0..j] in LDS, subdiagonal hn) is
// stored, the previous rotations applied, and a new complex Givens rotation
// [[conj(c), conj(s)], [-s, c]] (c = a/rho, s = b/rho) zeroes h_{j+1,j}; the
// rotated right-hand side e gives the residual norm |e_{j+1}|.  Called by
// one whole workgroup at the end of its kernel; thread 0 does the serial part.
__device__ __forceinline__ void givens_column(int j, int m, const double2 *h, double hn,
                                              double2 *H, double2 *cs, double2 *sn, double2 *e,
                                              GmresCtl *ctl) {
    double2 *col = H + (long)j * (m + 1);    // column-major, column j
    for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = h[i];
    __syncthreads();
    if (threadIdx.x != 0) return;
    col[j + 1] = cd(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        double2 a = col[i], b = col[i + 1];
        double2 c = cs[i], s = sn[i];
        double2 t = cadd(cmul(cd(c.x, -c.y), a), cmul(cd(s.x, -s.y), b));
        col[i + 1] = csub(cmul(c, b), cmul(s, a));
        col[i] = t;
    }
    double2 a = col[j];
    double den = sqrt(a.x * a.x + a.y * a.y + hn * hn);
    double2 c = den > 0 ? cd(a.x / den, a.y / den) : cd(1.0, 0.0);
    double2 s = den > 0 ? cd(hn / den, 0.0) : cd(0.0, 0.0);
    cs[j] = c;
    sn[j] = s;
    col[j] = cd(den, 0.0);
    col[j + 1] = cd(0.0, 0.0);
    double2 ej = e[j];
    e[j + 1] = cd(-(s.x * ej.x - s.y * ej.y), -(s.x * ej.y + s.y * ej.x));
    e[j] = cmul(cd(c.x, -c.y), ej);
    double res = sqrt(e[j + 1].x * e[j + 1].x + e[j + 1].y * e[j + 1].y);
    ctl->j = j + 1;
    ctl->resid = res;
    ctl->inv_hn = hn > 0 ? 1.0 / hn : 0.0;
    if (!isfinite(hn) || !isfinite(res)) { ctl->bad = 1; ctl->done = 1; return; }
    if (res <= ctl->tol * ctl->bnorm || hn == 0.0) { ctl->done = 1; ctl->conv = 1; }
}

// Column j from the two Gram-Schmidt passes' partials and ||w|| (one
// workgroup).
__global__ __launch_bounds__(256) void gmres_givens_kernel(int j, int m, const double2 *part1,
                                                           const double2 *part2, int nb,
                                                           const double *part, int np, double2 *H,
                                                           double2 *cs, double2 *sn, double2 *e,
                                                           GmresCtl *ctl) {
    if (ctl->done) return;
    __shared__ double2 h[256];
    // h_{i,j} = first-pass + second-pass projections, reduced over chunks
    reduce_dots(part1, nb, m + 1, j + 1, h, 0);
    reduce_dots(part2, nb, m + 1, j + 1, h, 1);
    double hn = sqrt(wave_reduce_parts(part, np));
    givens_column(j, m, h, hn, H, cs, sn, e, ctl);
}

// Fused Arnoldi step, after lh_matvec_reg_kernel<.., true>: the first-pass
// projections h1 reduced from the matvec's np partials, w <- w - V h1 over
// this chunk, then the chunk's partials of V^H w (second pass, part_out) and
// of |w|^2 (norm_part).  Workgroup 0 stores h1 as column j of H.
__global__ __launch_bounds__(256) void cgs_pass1_kernel(long n, const double2 *V, int nv,
                                                        const double2 *part_in, int np, int ld,
                                                        double2 *w, double2 *part_out,
                                                        double *norm_part, double2 *hcol,
                                                        const GmresCtl *ctl) {
    if (ctl->done) return;
    __shared__ double2 dots[256];
    __shared__ double red[4];
    reduce_parts_wide(part_in, np, ld, nv, dots);
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < nv; i += blockDim.x) hcol[i] = dots[i];
    long lo, hi;
    chunk_range(n, &lo, &hi);
    double s = 0.0;
    for (long el = lo + threadIdx.x; el < hi; el += blockDim.x) {
        double2 acc = cd(0.0, 0.0);
        for (int k = 0; k < nv; ++k) acc = cadd(acc, cmul(dots[k], V[(long)k * n + el]));
        double2 o = csub(w[el], acc);
        w[el] = o;
        s += o.x * o.x + o.y * o.y;
    }
    __syncthreads();   // this chunk of w is final (each element is read back by its writer)
    chunk_dots(n, V, nv, w, lo, hi, part_out, ld);
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) norm_part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Fused Arnoldi step, last kernel: the second-pass projections h2 from the
// nb partials; the new vector's norm from |w|^2 - |h2|^2 (w minus its
// projection on the orthonormal basis: the two are orthogonal, so their
// squared norms add up); w <- (w - V h2) / hn over this chunk, which makes
// w the next basis vector; workgroup 0 adds h2 to column j (h1, stored by
// cgs_pass1_kernel) and applies the rotations.
__global__ __launch_bounds__(256) void cgs_pass2_kernel(int j, int m, long n, const double2 *V,
                                                        double2 *w, const double2 *part2, int nb,
                                                        const double *norm_part, double2 *H,
                                                        double2 *cs, double2 *sn, double2 *e,
                                                        GmresCtl *ctl) {
    if (ctl->done) return;
    __shared__ double2 h2[256];
    const int nv = j + 1;
    reduce_parts_wide(part2, nb, m + 1, nv, h2);
    const double n1 = wave_reduce_parts(norm_part, nb);
    double s2 = 0.0;
    for (int k = 0; k < nv; ++k) s2 += h2[k].x * h2[k].x + h2[k].y * h2[k].y;
    const double hn2 = n1 - s2;
    const double hn = !isfinite(hn2) ? hn2 : (hn2 > 0.0 ? sqrt(hn2) : 0.0);
    const double inv = hn > 0.0 && isfinite(hn) ? 1.0 / hn : 0.0;
    long lo, hi;
    chunk_range(n, &lo, &hi);
    for (long el = lo + threadIdx.x; el < hi; el += blockDim.x) {
        double2 acc = cd(0.0, 0.0);
        for (int k = 0; k < nv; ++k) acc = cadd(acc, cmul(h2[k], V[(long)k * n + el]));
        w[el] = cscale(inv, csub(w[el], acc));
    }
    if (blockIdx.x != 0) return;
    __syncthreads();
    const double2 *col = H + (long)j * (m + 1);
    for (int i = threadIdx.x; i < nv; i += blockDim.x) h2[i] = cadd(col[i], h2[i]);
    __syncthreads();
    givens_column(j, m, h2, hn, H, cs, sn, e, ctl);
}

// End of a cycle: y = R^{-1} e over the ctl->j columns of the rotated
// Hessenberg matrix, then x += sum_k y_k V_k (multiaxpy_ctl) and the cycle is
// marked finished (gmres_mark).  require_done: only when the cycle has
// stopped (the speculative end enqueued right after the first chunk).
// One thread; ctl->skip tells the two following kernels to do nothing.
__global__ void gmres_backsolve_kernel(int m, const double2 *H, const double2 *e, double2 *y,
                                       GmresCtl *ctl, int require_done) {
    if (threadIdx.x != 0) return;
    if (ctl->finished || (require_done && !ctl->done)) {
        ctl->skip = 1;
        return;
    }
    ctl->skip = 0;
    int jd = ctl->j;
    for (int i = jd - 1; i >= 0; --i) {
        double2 t = e[i];
        for (int k = i + 1; k < jd; ++k) t = csub(t, cmul(H[(long)k * (m + 1) + i], y[k]));
        double2 d = H[(long)i * (m + 1) + i];
        y[i] = cmul(t, cinv(d));
    }
}

__global__ void multiaxpy_ctl_kernel(long n, const double2 *V, const double2 *h, double2 *w,
                                     const GmresCtl *ctl) {
    if (ctl->skip) return;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    int nv = ctl->j;
    double2 acc = cd(0.0, 0.0);
    for (int k = 0; k < nv; ++k) acc = cadd(acc, cmul(h[k], V[(long)k * n + e]));
    w[e] = cadd(w[e], acc);
}

__global__ void gmres_mark_kernel(GmresCtl *ctl) {
    if (threadIdx.x != 0 || ctl->skip) return;
    ctl->finished = 1;
    ctl->total += ctl->j;
}

// lh_matvec_kernel with an early exit for a finished cycle
__global__ __launch_bounds__(256) void lh_matvec_ctl_kernel(Phys P, const StripMeta *strips,
                                                            const double2 *LH, const double2 *x,
                                                            double2 *y, const GmresCtl *ctl) {
    if (ctl->done) return;
    lh_matvec_body(P, strips, LH, x, y, 1);
}

}  // namespace

static inline unsigned lh_grid(const Phys &P) {
    unsigned ntr = 2 * (P.nsub - 1), ntile = (P.ny + 3) / 4;
    return 8u * ntr * ((ntile + 7) / 8);
}

// Workgroups of one register-resident L_h kernel that fit on the device at
// once (queried once per kernel and process).
static int lh_resident(int nch, bool dots) {
    static int cache[2][2] = {{-1, -1}, {-1, -1}};
    const int a = nch <= 9 ? 0 : 1, b = dots ? 1 : 0;
    if (cache[a][b] < 0) {
        const void *fn = a == 0 ? (dots ? (const void *)lh_matvec_reg_kernel<9, 1, 2, true>
                                        : (const void *)lh_matvec_reg_kernel<9, 1, 2, false>)
                                : (dots ? (const void *)lh_matvec_reg_kernel<17, 1, 1, true>
                                        : (const void *)lh_matvec_reg_kernel<17, 1, 1, false>);
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0) != hipSuccess)
            return 512;
        cache[a][b] = max(1, per * cus);
    }
    return cache[a][b];
}

// Plan of the register-resident L_h kernel.  R = resident workgroups per
// row tile; class c with n_c of the N strips gets ceil(R n_c / N) strip
// groups (at least 1, at most n_c), so the resident slots are shared out in
// proportion to the strips and no group is empty.  Classes with the most
// strips per group come first in the dispatch order.
int lh_plan_build(int ny, int nsub, const int *strip_cls, int ncls, std::vector<LhClass> &tab,
                  std::vector<int> &list) {
    tab.clear();
    list.clear();
    const int nch = (ny + 63) / 64;
    if (nch > 17 || nsub < 1 || ncls < 1) return 0;
    const int tiles = (ny + 1) / 2;
    const int R = max(1, lh_resident(nch, true) / tiles);
    std::vector<std::vector<int>> members(ncls);
    for (int j = 0; j < nsub; ++j)
        if (strip_cls[j] >= 0 && strip_cls[j] < ncls) members[strip_cls[j]].push_back(j);
    std::vector<LhClass> cl;
    for (int c = 0; c < ncls; ++c) {
        const int cnt = (int)members[c].size();
        if (cnt == 0) continue;
        LhClass e;
        e.cls = c;
        e.count = cnt;
        e.groups = (int)std::min<long>(cnt, std::max<long>(1, ((long)R * cnt + nsub - 1) / nsub));
        e.list_off = 0;
        e.block_off = 0;
        cl.push_back(e);
    }
    std::stable_sort(cl.begin(), cl.end(), [](const LhClass &a, const LhClass &b) {
        return (a.count + a.groups - 1) / a.groups > (b.count + b.groups - 1) / b.groups;
    });
    long blocks = 0;
    for (LhClass &e : cl) {
        e.list_off = (int)list.size();
        list.insert(list.end(), members[e.cls].begin(), members[e.cls].end());
        e.block_off = (int)blocks;
        blocks += (long)tiles * e.groups;
        tab.push_back(e);
    }
    return blocks > INT32_MAX ? 0 : (int)blocks;
}

int lh_fused_blocks_bound(int ny, int nsub, int ncls) {
    const int nch = (ny + 63) / 64;
    if (nch > 17 || nsub < 1 || ncls < 1) return 0;
    const int tiles = (ny + 1) / 2;
    const int R = max(1, lh_resident(nch, true) / tiles);
    return tiles * min(nsub, R + ncls);
}

// L_h x (mode_p = 0) or x - L_h x (mode_p = 1); ctl may be null.  The
// register-resident kernel reuses every block row over the strips of its
// group; beyond 17 column chunks the row-per-wave kernel is used.  With
// part given (register-resident kernel only, mode_p = 1, x = V_{nv-1},
// nv <= 64) the first Gram-Schmidt pass's partials go to part.
static hipError_t lh_apply(hipStream_t st, const Phys &P, const StripMeta *strips, int ncls,
                           const LhPlan &pl, const double2 *LH, const double2 *x, double2 *y,
                           int mode_p, const GmresCtl *ctl, const double2 *V = nullptr,
                           long ng = 0, int nv = 0, double2 *part = nullptr, int ld = 0) {
    if (pl.md.phi) {
        if (part) return hipErrorInvalidValue;
        return launch_lh_modal(st, P, strips, pl.md, x, y, mode_p, ctl);
    }
    int nch = (P.ny + 63) / 64;
    const bool reg = nch <= 17 && pl.blocks > 0 && pl.tab && pl.list &&
                     pl.tiles == (P.ny + 1) / 2;
    if (part && (!reg || mode_p != 1 || nv < 1 || nv > 64 || !V))
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)pl.blocks);
    if (reg && nch <= 9) {
        if (part)
            hipLaunchKernelGGL((lh_matvec_reg_kernel<9, 1, 2, true>), grid, dim3(256), 0, st, P,
                               pl.tab, pl.ncls, pl.list, pl.tiles, LH, x, y, mode_p, ctl, V, ng,
                               nv, part, ld);
        else
            hipLaunchKernelGGL((lh_matvec_reg_kernel<9, 1, 2, false>), grid, dim3(256), 0, st, P,
                               pl.tab, pl.ncls, pl.list, pl.tiles, LH, x, y, mode_p, ctl, V, ng,
                               nv, part, ld);
    } else if (reg) {
        if (part)
            hipLaunchKernelGGL((lh_matvec_reg_kernel<17, 1, 1, true>), grid, dim3(256), 0, st, P,
                               pl.tab, pl.ncls, pl.list, pl.tiles, LH, x, y, mode_p, ctl, V, ng,
                               nv, part, ld);
        else
            hipLaunchKernelGGL((lh_matvec_reg_kernel<17, 1, 1, false>), grid, dim3(256), 0, st, P,
                               pl.tab, pl.ncls, pl.list, pl.tiles, LH, x, y, mode_p, ctl, V, ng,
                               nv, part, ld);
    } else if (ctl) {
        hipLaunchKernelGGL(lh_matvec_ctl_kernel, dim3(lh_grid(P)), dim3(256), 0, st, P, strips, LH,
                           x, y, ctl);
    } else {
        hipLaunchKernelGGL(lh_matvec_kernel, dim3(lh_grid(P)), dim3(256), 0, st, P, strips, LH, x,
                           y, mode_p);
    }
    return hipGetLastError();
}

int gmres_chunks(long n) {
    long nb = (n + 255) / 256;
    return (int)(nb < 256 ? nb : 256);
}

hipError_t launch_gmres_iteration(hipStream_t st, const Phys &P, const StripMeta *strips,
                                  int ncls, const LhPlan &pl, const double2 *LH, long n, int j,
                                  int m, double2 *V, double2 *part1, double2 *part2,
                                  double *norm_part, double2 *H, double2 *cs, double2 *sn,
                                  double2 *e, GmresCtl *ctl, double2 *mvpart) {
    double2 *vj = V + (long)j * n, *w = V + (long)(j + 1) * n;
    unsigned nb = (unsigned)gmres_chunks(n);
    unsigned ne = (unsigned)((n + 255) / 256);
    int ld = m + 1;
    const int np1 = pl.blocks;
    if (mvpart && np1 > 0 && j + 1 <= 64) {
        // three kernels: matvec with the first pass's partials, first update
        // with the second pass's partials, second update with normalisation
        // and rotation
        hipError_t er = lh_apply(st, P, strips, ncls, pl, LH, vj, w, 1, ctl, V, n, j + 1, mvpart,
                                 ld);
        if (er != hipSuccess) return er;
        hipLaunchKernelGGL(cgs_pass1_kernel, dim3(nb), dim3(256), 0, st, n, (const double2 *)V,
                           j + 1, (const double2 *)mvpart, np1, ld, w, part2, norm_part,
                           H + (long)j * ld, (const GmresCtl *)ctl);
        hipLaunchKernelGGL(cgs_pass2_kernel, dim3(nb), dim3(256), 0, st, j, m, n,
                           (const double2 *)V, w, (const double2 *)part2, (int)nb,
                           (const double *)norm_part, H, cs, sn, e, ctl);
        return hipGetLastError();
    }
    hipError_t er = lh_apply(st, P, strips, ncls, pl, LH, vj, w, 1, ctl);
    if (er != hipSuccess) return er;
    hipLaunchKernelGGL(cgs_dots_kernel, dim3(nb), dim3(256), 0, st, n, V, j + 1, w, part1, ld,
                       ctl);
    hipLaunchKernelGGL(cgs_update_kernel, dim3(nb), dim3(256), 0, st, n, V, j + 1, part1,
                       (int)nb, ld, w, part2, (double *)nullptr, ctl);
    hipLaunchKernelGGL(cgs_update_kernel, dim3(nb), dim3(256), 0, st, n, V, j + 1, part2,
                       (int)nb, ld, w, (double2 *)nullptr, norm_part, ctl);
    hipLaunchKernelGGL(gmres_givens_kernel, dim3(1), dim3(256), 0, st, j, m, part1, part2,
                       (int)nb, norm_part, (int)nb, H, cs, sn, e, ctl);
    hipLaunchKernelGGL(scale_ctl_kernel, dim3(ne), dim3(256), 0, st, n, w, w, ctl);
    return hipGetLastError();
}

hipError_t launch_gmres_begin(hipStream_t st, long n, const double2 *r, double *norm_part,
                              int first, double accept, double2 *V0, double2 *e, int m,
                              GmresCtl *ctl, const StepCtl *sctl) {
    unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(norm_partials_kernel, dim3(nb), dim3(256), 0, st, n, r, norm_part);
    hipLaunchKernelGGL(gmres_begin_kernel, dim3(1), dim3(64), 0, st, norm_part, (int)nb, first,
                       accept, e, m, ctl, sctl);
    hipLaunchKernelGGL(scale_ctl_kernel, dim3(nb), dim3(256), 0, st, n, r, V0, ctl);
    return hipGetLastError();
}

hipError_t launch_gmres_finish(hipStream_t st, long n, int m, const double2 *H, const double2 *e,
                               double2 *y, const double2 *V, double2 *x, GmresCtl *ctl,
                               int require_done) {
    hipLaunchKernelGGL(gmres_backsolve_kernel, dim3(1), dim3(64), 0, st, m, H, e, y, ctl,
                       require_done);
    hipLaunchKernelGGL(multiaxpy_ctl_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       n, V, y, x, ctl);
    hipLaunchKernelGGL(gmres_mark_kernel, dim3(1), dim3(64), 0, st, ctl);
    return hipGetLastError();
}

hipError_t launch_lh_matvec(hipStream_t st, const Phys &P, const StripMeta *strips, int ncls,
                            const LhPlan &pl, const double2 *LH, const double2 *x, double2 *y,
                            int mode_p) {
    return lh_apply(st, P, strips, ncls, pl, LH, x, y, mode_p, nullptr);
}

hipError_t launch_multidot(hipStream_t st, long n, const double2 *V, int nv, const double2 *w,
                           double2 *part, int nblk) {
    hipLaunchKernelGGL(multidot_kernel, dim3(nblk), dim3(256), 0, st, n, V, nv, w, part);
    return hipGetLastError();
}

hipError_t launch_multidot_finalize(hipStream_t st, const double2 *part, int nv, int nblk,
                                    double2 *out) {
    hipLaunchKernelGGL(multidot_finalize_kernel, dim3(1), dim3(256), 0, st, part, nv, nblk, out);
    return hipGetLastError();
}

hipError_t launch_multiaxpy(hipStream_t st, long n, const double2 *V, int nv, const double2 *h,
                            double2 *w, int sub) {
    hipLaunchKernelGGL(multiaxpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                       V, nv, h, w, sub);
    return hipGetLastError();
}

hipError_t launch_norm_partials(hipStream_t st, long n, const double2 *x, double *part, int nblk) {
    hipLaunchKernelGGL(norm_partials_kernel, dim3(nblk), dim3(256), 0, st, n, x, part);
    return hipGetLastError();
}

hipError_t launch_scale_copy(hipStream_t st, long n, const double2 *x, double2 s, double2 *y) {
    hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                       x, s, y);
    return hipGetLastError();
}

hipError_t launch_axpby(hipStream_t st, long n, double2 a, const double2 *x, double2 b,
                        const double2 *y, double2 *z) {
    hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a,
                       x, b, y, z);
    return hipGetLastError();
}
