// Block-Thomas factorisation of the strip operators with dense ny x ny
// Schur complements (the strip system of eq. NproblemRobinNL ordered by
// x node-lines is block tridiagonal with tridiagonal blocks; K_j is complex
// symmetric, so the sub-diagonal block L_i equals U_{i-1}^T):
//     S_0 = D_0,   S_i = D_i - U_{i-1}^T S_{i-1}^{-1} U_{i-1}
// from above, and in the twisted form used by the strip solve also
//     T_{nx-1} = D_{nx-1},   T_i = D_i - U_i T_{i+1}^{-1} U_i^T
// from below, meeting at a middle line that eliminates both neighbours.
// Each S_i is inverted in place by blocked Gauss-Jordan without pivoting:
// -i K_j has a positive definite Hermitian part (2/dt M + c p M^Gamma), so
// elimination without pivoting is well defined for every Schur complement.
// The rank-BK updates run as complex GEMMs on the matrix cores
// (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32, complex product as four
// real products on split real/imaginary tiles).
#include "osm_internal.h"

#define GJ_BK 32

namespace {

template <typename T> struct vec4_of;
template <> struct vec4_of<double> { typedef v4d type; };
template <> struct vec4_of<float> { typedef v4f type; };

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of the 16 x 16 accumulator held in element v of `lane`; the column is
// lane % 16.  The FP64 instruction spreads a lane's four rows with stride 4,
// the FP32 one keeps them consecutive.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int v);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int v) { return (lane >> 4) + 4 * v; }
template <> __device__ __forceinline__ int acc_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }

template <typename T2> __device__ __forceinline__ T2 mk2(double x, double y);
template <> __device__ __forceinline__ double2 mk2<double2>(double x, double y) { return cd(x, y); }
template <> __device__ __forceinline__ float2 mk2<float2>(double x, double y) {
    float2 r; r.x = (float)x; r.y = (float)y; return r;
}

// Schur complement of line lines[z], written into its factor slot:
//   D_i                                      kind 0 (first line of a chain)
//   - U_{i-1}^T F_{i-1} U_{i-1}              kind bit 0 (eliminated from above)
//   - U_i F_{i+1} U_i^T                      kind bit 1 (eliminated from below)
// where F_{i-1} and F_{i+1} already hold the inverses of the neighbouring
// lines' Schur complements.
template <typename T>
__global__ void schur_kernel(int n, typename cplx_of<T>::type *F, const int *lines,
                             const int *kind, const double2 *Dc, const double2 *Uc) {
    typedef typename cplx_of<T>::type T2;
    int z = blockIdx.z;
    int r = blockIdx.y * 16 + threadIdx.y;
    int c = blockIdx.x * 16 + threadIdx.x;
    if (r >= n || c >= n) return;
    long L = lines[z];
    int kd = kind[z];
    double2 val = cd(0.0, 0.0);
    if (abs(r - c) <= 1) val = Dc[(L * n + r) * 3 + (c - r + 1)];
    if (kd & 1) {
        long Lp = L - 1;
        const T2 *Sp = F + Lp * n * (long)n;
        for (int a = max(r - 1, 0); a <= min(r + 1, n - 1); ++a) {
            double2 uar = Uc[(Lp * n + a) * 3 + (r - a + 1)];        // U_{i-1}(a, r)
            double2 t = cd(0.0, 0.0);
            for (int b = max(c - 1, 0); b <= min(c + 1, n - 1); ++b) {
                double2 ubc = Uc[(Lp * n + b) * 3 + (c - b + 1)];    // U_{i-1}(b, c)
                T2 s = Sp[(long)a * n + b];
                t = cadd(t, cmul(cd(s.x, s.y), ubc));
            }
            val = csub(val, cmul(uar, t));
        }
    }
    if (kd & 2) {
        const T2 *Sn = F + (L + 1) * n * (long)n;
        for (int a = max(r - 1, 0); a <= min(r + 1, n - 1); ++a) {
            double2 ura = Uc[(L * n + r) * 3 + (a - r + 1)];         // U_i(r, a)
            double2 t = cd(0.0, 0.0);
            for (int b = max(c - 1, 0); b <= min(c + 1, n - 1); ++b) {
                double2 ucb = Uc[(L * n + c) * 3 + (b - c + 1)];     // U_i(c, b) = U_i^T(b, c)
                T2 s = Sn[(long)a * n + b];
                t = cadd(t, cmul(cd(s.x, s.y), ucb));
            }
            val = csub(val, cmul(ura, t));
        }
    }
    F[L * n * (long)n + (long)r * n + c] = mk2<T2>(val.x, val.y);
}

// One Gauss-Jordan pivot block step, panel part.  Block k covers rows and
// columns [k0, k0+b).  Every workgroup inverts the b x b pivot block P in LDS
// (redundantly), then
//   R[:, tile]  = P A[k-rows, tile]   (with R[:, k-cols] = P)
//   C'[tile, :] = A[tile, k-cols]     (with C'[k-rows, :] = -I)
// so that the whole update is one GEMM:  A <- A|masked - C' R, where the
// base drops block row k and block column k.
template <typename T>
__global__ __launch_bounds__(256) void gj_panel_kernel(int n, int kb,
                                                       const typename cplx_of<T>::type *F,
                                                       const int *lines,
                                                       typename cplx_of<T>::type *Rbuf,
                                                       typename cplx_of<T>::type *Cbuf) {
    typedef typename cplx_of<T>::type T2;
    int z = blockIdx.y, J = blockIdx.x;
    const T2 *A = F + (long)lines[z] * n * (long)n;
    int k0 = kb * GJ_BK;
    int b = min(GJ_BK, n - k0);
    __shared__ T Pr[GJ_BK][GJ_BK + 1], Pi[GJ_BK][GJ_BK + 1];
    __shared__ T Ar[GJ_BK][65], Ai[GJ_BK][65];
    int tid = threadIdx.x;
    for (int e = tid; e < GJ_BK * GJ_BK; e += 256) {
        int r = e / GJ_BK, c = e % GJ_BK;
        T2 v;
        if (r < b && c < b) v = A[(long)(k0 + r) * n + k0 + c];
        else { v.x = (r == c) ? (T)1 : (T)0; v.y = 0; }
        Pr[r][c] = v.x; Pi[r][c] = v.y;
    }
    for (int e = tid; e < GJ_BK * 64; e += 256) {
        int t = e / 64, cc = e % 64, col = J * 64 + cc;
        T2 v;
        if (t < b && col < n) v = A[(long)(k0 + t) * n + col];
        else { v.x = 0; v.y = 0; }
        Ar[t][cc] = v.x; Ai[t][cc] = v.y;
    }
    __syncthreads();
    // in-place Gauss-Jordan inversion of the b x b pivot block
    for (int p = 0; p < b; ++p) {
        T ar = Pr[p][p], ai = Pi[p][p];
        T den = ar * ar + ai * ai;
        T ivr = ar / den, ivi = -ai / den;
        T nv_r[4], nv_i[4];
        int cnt = 0;
        for (int e = tid; e < GJ_BK * GJ_BK; e += 256, ++cnt) {
            int r = e / GJ_BK, c = e % GJ_BK;
            T xr = Pr[r][c], xi = Pi[r][c];
            T yr, yi;
            if (r >= b || c >= b) { yr = xr; yi = xi; }
            else if (r == p && c == p) { yr = ivr; yi = ivi; }
            else if (r == p) { yr = ivr * xr - ivi * xi; yi = ivr * xi + ivi * xr; }
            else {
                T fr = Pr[r][p], fi = Pi[r][p];
                T gr = fr * ivr - fi * ivi, gi = fr * ivi + fi * ivr;     // A[r][p] / A[p][p]
                if (c == p) { yr = -gr; yi = -gi; }
                else {
                    T pr = Pr[p][c], pi = Pi[p][c];
                    yr = xr - (gr * pr - gi * pi);
                    yi = xi - (gr * pi + gi * pr);
                }
            }
            nv_r[cnt] = yr; nv_i[cnt] = yi;
        }
        __syncthreads();
        cnt = 0;
        for (int e = tid; e < GJ_BK * GJ_BK; e += 256, ++cnt) {
            int r = e / GJ_BK, c = e % GJ_BK;
            Pr[r][c] = nv_r[cnt]; Pi[r][c] = nv_i[cnt];
        }
        __syncthreads();
    }
    T2 *R = Rbuf + (long)z * GJ_BK * n;
    for (int e = tid; e < GJ_BK * 64; e += 256) {
        int t = e / 64, cc = e % 64, col = J * 64 + cc;
        if (t >= b || col >= n) continue;
        T vr = 0, vi = 0;
        if (col >= k0 && col < k0 + b) { vr = Pr[t][col - k0]; vi = Pi[t][col - k0]; }
        else {
            for (int s = 0; s < b; ++s) {
                T pr = Pr[t][s], pi = Pi[t][s], xr = Ar[s][cc], xi = Ai[s][cc];
                vr += pr * xr - pi * xi;
                vi += pr * xi + pi * xr;
            }
        }
        T2 o; o.x = vr; o.y = vi;
        R[(long)t * n + col] = o;
    }
    T2 *C = Cbuf + (long)z * n * GJ_BK;
    for (int e = tid; e < 64 * GJ_BK; e += 256) {
        int rr = e / GJ_BK, t = e % GJ_BK, row = J * 64 + rr;
        if (row >= n || t >= b) continue;
        T2 v;
        if (row >= k0 && row < k0 + b) { v.x = (row - k0 == t) ? (T)-1 : (T)0; v.y = 0; }
        else v = A[(long)row * n + k0 + t];
        C[(long)row * GJ_BK + t] = v;
    }
}

// D = base + sign * A B for complex matrices (row-major, interleaved re/im),
// 64 x 64 output tile per workgroup, 32 x 32 per wave as 2 x 2 blocks of
// 16 x 16 MFMA accumulators (split real / imaginary parts).
template <typename T>
__global__ __launch_bounds__(256) void zgemm_kernel(GemmArgs<T> g) {
    typedef typename cplx_of<T>::type T2;
    typedef typename vec4_of<T>::type V4;
    constexpr int BM = 64, BN = 64, BKK = 16;
    int z = blockIdx.z;
    int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const T2 *A = g.A + (long)z * g.strideA;
    const T2 *B = g.B + (long)z * g.strideB;
    long cdo = (long)(g.idxCD ? g.idxCD[z] : z) * g.strideCD;
    const T2 *C = g.C ? g.C + cdo : nullptr;
    T2 *D = g.D + cdo;
    int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    __shared__ T As_r[BM][BKK + 1], As_i[BM][BKK + 1];
    __shared__ T Bs_r[BKK][BN + 1], Bs_i[BKK][BN + 1];
    V4 acc_r[2][2], acc_i[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int row = m0 + wr + bi * 16 + acc_row<T>(lane, v);
                int col = n0 + wc + bj * 16 + (lane & 15);
                T br = 0, bim = 0;
                bool masked = (row >= g.mask_lo && row < g.mask_hi) ||
                              (col >= g.mask_lo && col < g.mask_hi);
                if (C && row < g.M && col < g.N && !masked) {
                    T2 t = C[(long)row * g.ldc + col];
                    br = t.x; bim = t.y;
                }
                acc_r[bi][bj][v] = br;
                acc_i[bi][bj][v] = bim;
            }
    T sg = (T)g.sign;
    for (int k0 = 0; k0 < g.K; k0 += BKK) {
        for (int e = tid; e < BM * BKK; e += 256) {
            int r = e / BKK, kk = e % BKK;
            T2 v;
            if (m0 + r < g.M && k0 + kk < g.K) v = A[(long)(m0 + r) * g.lda + k0 + kk];
            else { v.x = 0; v.y = 0; }
            As_r[r][kk] = sg * v.x;
            As_i[r][kk] = sg * v.y;
        }
        for (int e = tid; e < BKK * BN; e += 256) {
            int kk = e / BN, c = e % BN;
            T2 v;
            if (k0 + kk < g.K && n0 + c < g.N) v = B[(long)(k0 + kk) * g.ldb + n0 + c];
            else { v.x = 0; v.y = 0; }
            Bs_r[kk][c] = v.x;
            Bs_i[kk][c] = v.y;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BKK; ks += 4) {
            T a_r[2], a_i[2], b_r[2], b_i[2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) {
                a_r[bi] = As_r[wr + bi * 16 + (lane & 15)][ks + (lane >> 4)];
                a_i[bi] = As_i[wr + bi * 16 + (lane & 15)][ks + (lane >> 4)];
            }
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                b_r[bj] = Bs_r[ks + (lane >> 4)][wc + bj * 16 + (lane & 15)];
                b_i[bj] = Bs_i[ks + (lane >> 4)][wc + bj * 16 + (lane & 15)];
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    acc_r[bi][bj] = mfma16(a_r[bi], b_r[bj], acc_r[bi][bj]);
                    acc_r[bi][bj] = mfma16(-a_i[bi], b_i[bj], acc_r[bi][bj]);
                    acc_i[bi][bj] = mfma16(a_r[bi], b_i[bj], acc_i[bi][bj]);
                    acc_i[bi][bj] = mfma16(a_i[bi], b_r[bj], acc_i[bi][bj]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int row = m0 + wr + bi * 16 + acc_row<T>(lane, v);
                int col = n0 + wc + bj * 16 + (lane & 15);
                if (row < g.M && col < g.N) {
                    T2 o;
                    o.x = acc_r[bi][bj][v];
                    o.y = acc_i[bi][bj][v];
                    D[(long)row * g.ldd + col] = o;
                }
            }
}

// Y = scale * T X with T tridiagonal given by coef[r][d] = T(r, r+d-1), or
// Y = scale * T^T X when transpose != 0.  X, Y: n x n dense.
__global__ void tridiag_apply_kernel(int n, const double2 *coef, int transpose, double scale,
                                     const double2 *X, double2 *Y) {
    int r = blockIdx.y;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double2 acc = cd(0.0, 0.0);
    for (int a = max(r - 1, 0); a <= min(r + 1, n - 1); ++a) {
        double2 t = transpose ? coef[(long)a * 3 + (r - a + 1)] : coef[(long)r * 3 + (a - r + 1)];
        acc = cadd(acc, cmul(t, X[(long)a * n + c]));
    }
    Y[(long)r * n + c] = cscale(scale, acc);
}

// Y = scale * M1y as a dense n x n matrix (1-D Q1 mass in y: hy/6, 2hy/3,
// hy/3 at the two ends).
__global__ void set_tridiag_mass_kernel(int n, double hy, double scale, double2 *Y) {
    int r = blockIdx.y;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double v = 0.0;
    if (c == r) v = (r == 0 || r == n - 1) ? hy / 3.0 : 2.0 * hy / 3.0;
    else if (abs(c - r) == 1) v = hy / 6.0;
    Y[(long)r * n + c] = cd(scale * v, 0.0);
}

// out = (add_eye ? -I : 0) + i * coef_im * X
__global__ void lh_form_kernel(int n, const double2 *X, double coef_im, int add_eye,
                               double2 *out) {
    int r = blockIdx.y;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double2 x = X[(long)r * n + c];
    double2 o = cd(-coef_im * x.y, coef_im * x.x);
    if (add_eye && r == c) o.x -= 1.0;
    out[(long)r * n + c] = o;
}

template <typename T>
__global__ void convert_kernel(long n, const double2 *src, typename cplx_of<T>::type *dst) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long stride = (long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        double2 v = src[i];
        dst[i] = mk2<typename cplx_of<T>::type>(v.x, v.y);
    }
}

}  // namespace

template <typename T>
hipError_t launch_schur(hipStream_t st, int n, typename cplx_of<T>::type *F, const int *lines,
                        const int *kind, int batch, const double2 *Dc, const double2 *Uc) {
    dim3 grid((n + 15) / 16, (n + 15) / 16, batch);
    hipLaunchKernelGGL(schur_kernel<T>, grid, dim3(16, 16), 0, st, n, F, lines, kind, Dc, Uc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gj_panel(hipStream_t st, int n, int kb, const typename cplx_of<T>::type *F,
                           const int *lines, int batch, typename cplx_of<T>::type *Rbuf,
                           typename cplx_of<T>::type *Cbuf) {
    dim3 grid((n + 63) / 64, batch);
    hipLaunchKernelGGL(gj_panel_kernel<T>, grid, dim3(256), 0, st, n, kb, F, lines, Rbuf, Cbuf);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zgemm(hipStream_t st, const GemmArgs<T> &g, int batch) {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, batch);
    hipLaunchKernelGGL(zgemm_kernel<T>, grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_convert(hipStream_t st, long n, const double2 *src, typename cplx_of<T>::type *dst) {
    long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(convert_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_tridiag_apply(hipStream_t st, int n, const double2 *coef, int transpose,
                                double scale, const double2 *X, double2 *Y) {
    hipLaunchKernelGGL(tridiag_apply_kernel, dim3((n + 255) / 256, n), dim3(256), 0, st, n, coef,
                       transpose, scale, X, Y);
    return hipGetLastError();
}

hipError_t launch_set_tridiag_mass(hipStream_t st, int n, double hy, double scale, double2 *Y) {
    hipLaunchKernelGGL(set_tridiag_mass_kernel, dim3((n + 255) / 256, n), dim3(256), 0, st, n, hy,
                       scale, Y);
    return hipGetLastError();
}

hipError_t launch_lh_form(hipStream_t st, int n, const double2 *X, double coef_im, int add_eye,
                          double2 *out) {
    hipLaunchKernelGGL(lh_form_kernel, dim3((n + 255) / 256, n), dim3(256), 0, st, n, X, coef_im,
                       add_eye, out);
    return hipGetLastError();
}

template hipError_t launch_schur<double>(hipStream_t, int, double2 *, const int *, const int *,
                                         int, const double2 *, const double2 *);
template hipError_t launch_schur<float>(hipStream_t, int, float2 *, const int *, const int *,
                                        int, const double2 *, const double2 *);
template hipError_t launch_gj_panel<double>(hipStream_t, int, int, const double2 *, const int *,
                                            int, double2 *, double2 *);
template hipError_t launch_gj_panel<float>(hipStream_t, int, int, const float2 *, const int *,
                                           int, float2 *, float2 *);
template hipError_t launch_zgemm<double>(hipStream_t, const GemmArgs<double> &, int);
template hipError_t launch_zgemm<float>(hipStream_t, const GemmArgs<float> &, int);
template hipError_t launch_convert<double>(hipStream_t, long, const double2 *, double2 *);
template hipError_t launch_convert<float>(hipStream_t, long, const double2 *, float2 *);
