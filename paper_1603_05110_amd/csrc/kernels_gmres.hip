// Interface-space kernels of the preconditioned algorithm (Section 3,
// eq. Lmpi; Section 4.2): the block matrix-vector product with L_h and the
// vector primitives of GMRES on P x = y, P = I - L_h.  FP64.
#include "osm_internal.h"

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Row a of output trace t of L_h x (eq. Lmpi): trace 2i (new r_i) is fed by
// strip i+1 through X^{i+1,1} l_{i+1} + X^{i+1,2} r_{i+1}; trace 2i+1 (new
// l_{i+1}) by strip i through X^{i,3} l_i + X^{i,4} r_i.  LH holds, per
// block set, the four dense blocks X^{.,1..4} (row-major ny x ny).
// mode_p = 1: y = x - L_h x (the preconditioner P), else y = L_h x.
__global__ __launch_bounds__(256) void lh_matvec_kernel(Phys P, const StripMeta *strips,
                                                        const double2 *LH, const double2 *x,
                                                        double2 *y, int mode_p) {
    int t = blockIdx.y;
    int n = P.ny;
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int a = blockIdx.x * 4 + wave;
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

}  // namespace

hipError_t launch_lh_matvec(hipStream_t st, const Phys &P, const StripMeta *strips,
                            const double2 *LH, const double2 *x, double2 *y, int mode_p) {
    dim3 grid((P.ny + 3) / 4, 2 * (P.nsub - 1));
    hipLaunchKernelGGL(lh_matvec_kernel, grid, dim3(256), 0, st, P, strips, LH, x, y, mode_p);
    return hipGetLastError();
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
