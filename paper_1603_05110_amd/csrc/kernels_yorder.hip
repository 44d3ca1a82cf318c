// Strip factor and solve in y-line order (the unknowns of a strip taken
// y-line by y-line): the strip matrix K_j is block tridiagonal with
// (nx x nx) blocks, nx = the strip's node-lines, ny blocks along y,
//     K = tridiag(B_{a-1}^T, A_a, B_a),
// A_a (within y-line a) and B_a (y-line a to a+1) both tridiagonal in x;
// K_j is complex symmetric, so the block below the diagonal is B^T.  The
// entries are those of the node-line coefficients (Dc(l, a, d) = K[(l, a),
// (l, a + d - 1)], Uc(l, a, d) = K[(l, a), (l + 1, a + d - 1)]):
//     A_a[l][l] = Dc(l, a, 1),  A_a[l][l+1] = A_a[l+1][l] = Uc(l, a, 1),
//     B_a[l][l] = Dc(l, a, 2),  B_a[l][l+1] = Uc(l, a, 2),
//     B_a[l+1][l] = K[(l+1, a), (l, a+1)] = Uc(l, a+1, 0).
// The block Thomas algorithm runs twisted: y-lines below the middle line
// m = (ny - 1) / 2 are eliminated from a = 0 up (T_a = A_a - B_{a-1}^T
// T_{a-1}^{-1} B_{a-1}), those above from a = ny - 1 down (U_a = A_a - B_a
// U_{a+1}^{-1} B_a^T), and the middle line takes both terms.  The stored
// factor is the inverse of every complement (nx x nx), nx^2 per y-line
// instead of the ny^2 per node-line of the node-line order.  The complements
// are formed and inverted in FP64; the inverses are stored in FP64, or in
// complex FP32 for the complex-FP32-with-refinement precision (the solve
// then multiplies in FP64 by rounded inverses, and the FP64 residual of the
// fixed point refines, as with the node-line order's FP32 factors).  The
// complements are complex symmetric with a positive-definite imaginary part
// (that of K_j, 2/dt M + c p M^Gamma, is; z^* S z for a Schur complement S
// equals w^* K w for a w whose last block is z), so Gauss-Jordan needs no
// pivoting; the stored inverses are symmetric up to rounding, and the solve
// reads them by columns.
//
// The sweeps are sequential in y, so both the factor and the solve are
// latency-bound chains, one per strip half: the factor keeps each
// complement in registers (one barrier per pivot), the solve keeps the data
// of the next few y-lines in flight in registers while it works on the
// current one.
#include "osm_internal.h"

#include <algorithm>
#include <type_traits>
#include <utility>

namespace {

__device__ __forceinline__ double2 yz() { return cd(0.0, 0.0); }
// the solve kernels return at once when the fixed point is done (as the
// node-line solve does)
__device__ __forceinline__ bool yidle(const StepCtl *c) {
    return c && (c->q_conv || c->k_done || c->bad);
}
__device__ __forceinline__ double2 ymul(double2 a, double2 b) {
    return cd(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 yfma(double2 a, double2 b, double2 c) {
    return cd(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 yneg(double2 a) { return cd(-a.x, -a.y); }
// stored inverse entries: FP64 or complex FP32, used in FP64.  A complex
// FP32 block keeps its rows at an even stride (the last column of an odd
// order padded with zero) so that the solve reads whole 16-byte pairs.
template <typename E>
__host__ __device__ constexpr int yld(int n) { return sizeof(E) == 8 ? (n + 1) & ~1 : n; }
__device__ __forceinline__ double2 y2d(double2 v) { return v; }
__device__ __forceinline__ double2 y2d(float2 v) { return cd((double)v.x, (double)v.y); }
__device__ __forceinline__ void yput(double2 *p, double2 v) { *p = v; }
__device__ __forceinline__ void yput(float2 *p, double2 v) {
    *p = make_float2((float)v.x, (float)v.y);
}
// c ? a : b, component-wise (a conditional on the struct itself selects
// between addresses and keeps the values out of registers)
__device__ __forceinline__ double2 ysel(bool c, double2 a, double2 b) {
    return cd(c ? a.x : b.x, c ? a.y : b.y);
}

// ---------------------------------------------------------------- factor
// A workgroup of 256 threads per strip half works on the complement padded
// with the identity to NP = 16 T >= nx (T = 2, 3 or 4, a template
// parameter).  Thread (tr, tc) = (tid >> 4, tid & 15) owns the entries
// (tr + 16 a, tc + 16 c), a, c < T, in registers.  The padding keeps the
// identity through the coupling products (its coefficients are zero) and
// through the inversion (it is decoupled).
constexpr int YF_THREADS = 256;

template <int T>
struct YFLds {
    static constexpr int NP = 16 * T;
    double2 *cb;      // 5 NP: A's diagonal and off-diagonal, B's diagonal, upper, lower
                      // (zero past n)
    double2 *gl;      // NP x NP: the previous inverse, then the product H
    double2 *rowsP;   // 2 x 8 x NP: the block step's pivot rows (by step parity)
    double2 *colsP;   // 2 x NP x 8: its pivot columns
    double2 *zs;      // 2 x 8 x NP: Z = D C_PR, and D on the pivot columns
    double2 *ds;      // 4 x 64: each wave's copy of D
};
template <int T>
__device__ __forceinline__ YFLds<T> yf_lds(double2 *base) {
    constexpr int NP = 16 * T;
    YFLds<T> L;
    L.cb = base;
    L.gl = L.cb + 5 * NP;
    L.rowsP = L.gl + NP * NP;
    L.colsP = L.rowsP + 16 * NP;
    L.zs = L.colsP + 16 * NP;
    L.ds = L.zs + 16 * NP;
    return L;
}
__host__ __device__ constexpr int yf_lds_count(int np) { return np * np + 53 * np + 256; }

// The coefficients one thread (row l = min(tid, n - 1)) contributes to
// y-line a's LDS copy: A's diagonal and off-diagonal, and B_ab's diagonal,
// upper and lower entries.  Loaded unconditionally (ab clamped to 0 when
// there is no coupling block) so that the next y-line's loads can be in
// flight while the current one is inverted; put() applies the masks and
// also writes B_ab y-line-major to YB for the solve.
struct YCoef { double2 ad, ao, bd, bu, bl; };
__device__ __forceinline__ YCoef yf_coef_load(const YStrip &S, int ny, int a, int ab,
                                              const double2 *Dc, const double2 *Uc) {
    YCoef q;
    const int l = min((int)threadIdx.x, S.nx - 1), abc = max(ab, 0);
    const long r = ((long)(S.off + l) * ny + a) * 3, rb = ((long)(S.off + l) * ny + abc) * 3;
    q.ad = Dc[r + 1];
    q.ao = Uc[r + 1];
    q.bd = Dc[rb + 2];
    q.bu = Uc[rb + 2];
    q.bl = Uc[rb + 3];    // Uc(l, ab + 1, 0)
    return q;
}
__device__ __forceinline__ void yf_coef_put(const YCoef &q, const YStrip &S, int ab, int np,
                                            double2 *cb, double2 *YB) {
    const int n = S.nx, l = threadIdx.x;
    if (l >= n) return;
    const bool in = l + 1 < n;
    cb[l] = q.ad;
    cb[np + l] = ysel(in, q.ao, yz());
    if (ab >= 0) {
        const double2 up = ysel(in, q.bu, yz()), lo = ysel(in, q.bl, yz());
        cb[2 * np + l] = q.bd;
        cb[3 * np + l] = up;
        cb[4 * np + l] = lo;
        double2 *yb = YB + S.boff + (long)ab * 3 * n;
        yb[l] = q.bd;
        yb[n + l] = up;
        yb[2 * n + l] = lo;
    }
}

// The entries index j contributes to the tridiagonal products, for its
// neighbours j - 1, j, j + 1: lower (tr = 0) B[j-1][j], B[j][j], B[j+1][j];
// upper (tr = 1) B[j][j-1], B[j][j], B[j][j+1]; zero outside [0, n).
struct Tri { double2 m1, z0, p1; };
__device__ __forceinline__ Tri yf_tri(const double2 *cb, int np, int j, int tr) {
    Tri t;
    const double2 *up = cb + 3 * np, *lo = cb + 4 * np;
    const int jm = max(j - 1, 0), jp = min(j, np - 1);
    t.z0 = cb[2 * np + j];
    t.m1 = ysel(j > 0, ysel(tr, lo[jm], up[jm]), yz());
    t.p1 = ysel(j + 1 < np, ysel(tr, up[jp], lo[jp]), yz());
    return t;
}

// A_a (padded with the identity) at (i, k) from cb
__device__ __forceinline__ double2 yf_a(const double2 *cb, int np, int n, int i, int k) {
    if (i >= n || k >= n) return cd(i == k ? 1.0 : 0.0, 0.0);
    const double2 dg = cb[i], od = cb[np + min(i, k)];
    return ysel(i == k, dg, ysel(k == i + 1 || i == k + 1, od, yz()));
}

// c -= (X G Y) with G in L.gl: lower C -= B^T G B, upper C -= B G B^T, as
// H = G Y (3 terms) then X H (3 terms); the coefficients past the padding
// edge are zero, so the reads are clamped.  Ends with L.gl free.
template <int T>
__device__ __forceinline__ void yf_sandwich(double2 (&c)[T][T], const YFLds<T> &L, int tr,
                                            int tc, int side) {
    constexpr int NP = 16 * T;
    double2 h[T][T];
#pragma unroll
    for (int cc = 0; cc < T; ++cc) {
        const int k = tc + 16 * cc;
        const Tri tk = yf_tri(L.cb, NP, k, side);
        const int km = max(k - 1, 0), kp = min(k + 1, NP - 1);
#pragma unroll
        for (int a = 0; a < T; ++a) {
            const double2 *gi = L.gl + (tr + 16 * a) * NP;
            h[a][cc] = yfma(gi[kp], tk.p1, yfma(gi[km], tk.m1, ymul(gi[k], tk.z0)));
        }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int cc = 0; cc < T; ++cc) L.gl[(tr + 16 * a) * NP + tc + 16 * cc] = h[a][cc];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < T; ++a) {
        const int i = tr + 16 * a;
        const Tri ti = yf_tri(L.cb, NP, i, side);
        const int im = max(i - 1, 0), ip = min(i + 1, NP - 1);
#pragma unroll
        for (int cc = 0; cc < T; ++cc) {
            const int k = tc + 16 * cc;
            const double2 s = yfma(ti.p1, L.gl[ip * NP + k],
                                   yfma(ti.m1, L.gl[im * NP + k], ymul(ti.z0, L.gl[i * NP + k])));
            c[a][cc].x -= s.x;
            c[a][cc].y -= s.y;
        }
    }
    __syncthreads();
}

// 1 / x for the pivots' squared moduli (positive, far from overflow and
// underflow): the hardware reciprocal refined by two Newton steps, a shorter
// dependent chain than the IEEE division with its scaling and fix-up steps.
__device__ __forceinline__ double yrcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
}

__device__ __forceinline__ double2 yshfl(double2 v, int src) {
    return cd(__shfl(v.x, src), __shfl(v.y, src));
}

// One block step S of the in-place Gauss-Jordan inversion (no pivoting):
// pivot block P = rows and columns 8 S .. 8 S + 7 (row group half S & 1,
// register slot S >> 1, known at compile time).  With D = C_PP^{-1}:
//     C_PP <- D,  C_PR <- D C_PR,  C_RP <- -C_RP D,  C_RR <- C_RR - C_RP D C_PR.
// The block's rows and columns go to LDS (buffers of the step's parity, so
// the next step needs no barrier before publishing); every wave inverts the
// 8 x 8 pivot block in its own lanes (lane 8 a + c holds D[a][c]; scalar
// Gauss-Jordan with lane shuffles, no pivoting); Z = D C_PR (D itself on
// the pivot columns) goes to LDS; each entry then takes 8 complex
// multiply-adds.  Two barriers per block step.
// The in-place Gauss-Jordan inversion (no pivoting) in block steps s =
// 0 .. 2T-1 of 8 pivots: P = rows and columns 8 s .. 8 s + 7.  With
// D = C_PP^{-1}:
//     C_PP <- D,  C_PR <- D C_PR,  C_RP <- -C_RP D,  C_RR <- C_RR - C_RP D C_PR.
// The register tile is rotated by one slot in rows and columns after every
// second step, so the pivot block always sits in slot 0 (row group half
// s & 1): slot a holds rows tr + 16 ((a + s/2) mod T), likewise the columns,
// and T rotations over the 2T steps restore the order.  Each step puts its
// pivot rows and columns in LDS (buffers of the step's parity, so the next
// step needs no barrier before publishing); every wave inverts the 8 x 8
// pivot block in its own lanes (lane 8 a + c holds D[a][c]; scalar
// Gauss-Jordan with lane shuffles); Z = D C_PR (D itself on the pivot
// columns) goes to LDS; each entry then takes 8 complex multiply-adds, as
// two rank-4 halves.  Two barriers per step.
template <int T>
__device__ __forceinline__ void yf_invert(double2 (&c)[T][T], const YFLds<T> &L, int tr, int tc) {
    constexpr int NP = 16 * T;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ar = lane >> 3, ac = lane & 7;
    double2 *dsw = L.ds + wave * 64;
#pragma unroll 1
    for (int s = 0; s < 2 * T; ++s) {
        const int hf = s & 1, p0 = 8 * s, rot = s >> 1;
        double2 *rowsP = L.rowsP + hf * 8 * NP, *colsP = L.colsP + hf * NP * 8;
        double2 *zs = L.zs + hf * 8 * NP;
        auto row_of = [&](int a) { return tr + 16 * ((a + rot) % T); };
        auto col_of = [&](int cc) { return tc + 16 * ((cc + rot) % T); };
        const bool prow = (tr >> 3) == hf, pcol = (tc >> 3) == hf;
        if (prow) {
#pragma unroll
            for (int cc = 0; cc < T; ++cc) rowsP[(tr & 7) * NP + col_of(cc)] = c[0][cc];
        }
        if (pcol) {
#pragma unroll
            for (int a = 0; a < T; ++a) colsP[row_of(a) * 8 + (tc & 7)] = c[a][0];
        }
        __syncthreads();
        // D = C_PP^{-1}, every wave on its own
        double2 D = rowsP[ar * NP + p0 + ac];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double2 pq = cd(lane_f64(D.x, 9 * q), lane_f64(D.y, 9 * q));
            const double inv = yrcp(pq.x * pq.x + pq.y * pq.y);
            const double2 d = cd(pq.x * inv, -pq.y * inv);
            const double2 rq = yshfl(D, 8 * q + ac), cq = yshfl(D, 8 * ar + q);
            const bool kq = ac == q;
            const double2 mu = ysel(kq, d, ymul(rq, d));
            const double sv = kq ? 0.0 : 1.0;
            const double2 nv = cd(fma(sv, D.x, fma(cq.y, mu.y, -cq.x * mu.x)),
                                  fma(sv, D.y, -fma(cq.x, mu.y, cq.y * mu.x)));
            D = ysel(ar == q, mu, nv);
        }
        dsw[lane] = D;
        // Z = D C_PR over all NP columns (D on the pivot columns)
#pragma unroll
        for (int w = 0; w < (8 * NP + 255) / 256; ++w) {
            const int v = (int)threadIdx.x + 256 * w;
            if (v < 8 * NP) {
                const int m = v / NP, k = v % NP;
                double2 z = yz();
#pragma unroll
                for (int l = 0; l < 8; ++l) z = yfma(dsw[m * 8 + l], rowsP[l * NP + k], z);
                const bool kp = k >= p0 && k < p0 + 8;
                zs[m * NP + k] = ysel(kp, dsw[m * 8 + min(max(k - p0, 0), 7)], z);
            }
        }
        __syncthreads();
        double2 acc[T][T];
#pragma unroll
        for (int a = 0; a < T; ++a)
#pragma unroll
            for (int cc = 0; cc < T; ++cc) acc[a][cc] = yz();
#pragma unroll
        for (int mh = 0; mh < 8; mh += 4) {
            double2 zk[T][4], cp[T][4];
#pragma unroll
            for (int cc = 0; cc < T; ++cc)
#pragma unroll
                for (int m = 0; m < 4; ++m) zk[cc][m] = zs[(mh + m) * NP + col_of(cc)];
#pragma unroll
            for (int a = 0; a < T; ++a)
#pragma unroll
                for (int m = 0; m < 4; ++m) cp[a][m] = colsP[row_of(a) * 8 + mh + m];
#pragma unroll
            for (int a = 0; a < T; ++a)
#pragma unroll
                for (int cc = 0; cc < T; ++cc)
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        acc[a][cc] = yfma(cp[a][m], zk[cc][m], acc[a][cc]);
        }
#pragma unroll
        for (int a = 0; a < T; ++a) {
#pragma unroll
            for (int cc = 0; cc < T; ++cc) {
                // the pivot columns start from zero (C_RP <- -C_RP D)
                const double2 base = cc == 0 ? ysel(pcol, yz(), c[a][cc]) : c[a][cc];
                const double2 nv = cd(base.x - acc[a][cc].x, base.y - acc[a][cc].y);
                // the pivot rows take Z (D C_PR, and D on the pivot columns)
                c[a][cc] = a == 0 ? ysel(prow, zs[(tr & 7) * NP + col_of(cc)], nv) : nv;
            }
        }
        if (hf == 1) {   // the next block's rows and columns into slot 0
            double2 t[T][T];
#pragma unroll
            for (int a = 0; a < T; ++a)
#pragma unroll
                for (int cc = 0; cc < T; ++cc) t[a][cc] = c[(a + 1) % T][(cc + 1) % T];
#pragma unroll
            for (int a = 0; a < T; ++a)
#pragma unroll
                for (int cc = 0; cc < T; ++cc) c[a][cc] = t[a][cc];
        }
    }
    __syncthreads();
}

template <int T, typename E>
__device__ __forceinline__ void yf_store(const double2 (&c)[T][T], E *out, int n, int tr,
                                         int tc) {
    const int ld = yld<E>(n);   // ld <= NP: an odd n is below NP
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int cc = 0; cc < T; ++cc) {
            const int i = tr + 16 * a, k = tc + 16 * cc;
            if (i < n && k < ld) yput(out + i * ld + k, k < n ? c[a][cc] : yz());
        }
}

template <int T>
__device__ __forceinline__ void yf_init(const YFLds<T> &L) {
    constexpr int NP = 16 * T;
    for (int e = threadIdx.x; e < 5 * NP; e += blockDim.x) L.cb[e] = yz();
}

// The two halves of every strip: blockIdx.x = 2 j + half.
template <int T, typename E>
__global__ __launch_bounds__(YF_THREADS) void yfactor_half_kernel(const YStrip *ys, int ny,
                                                                  const double2 *Dc,
                                                                  const double2 *Uc, E *YF,
                                                                  double2 *YB) {
    constexpr int NP = 16 * T;
    const int j = blockIdx.x >> 1, half = blockIdx.x & 1;
    const YStrip S = ys[j];
    const int n = S.nx, nn = n * yld<E>(n), m = (ny - 1) / 2;
    extern __shared__ double2 ylds[];
    const YFLds<T> L = yf_lds<T>(ylds);
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    yf_init(L);
    double2 c[T][T];
    const int a0 = half == 0 ? 0 : ny - 1, a1 = m, da = half == 0 ? 1 : -1;
    // coupling block of y-line a: lower B_{a-1}, upper B_a (none for a0)
    auto ab_of = [&](int a) { return a == a0 ? -1 : (half == 0 ? a - 1 : a); };
    YCoef nxt = yf_coef_load(S, ny, a0, -1, Dc, Uc);
    __syncthreads();
    for (int a = a0; a != a1; a += da) {
        const bool first = a == a0;
        const int ab = ab_of(a);
        if (!first) {   // the previous inverse, for the product
#pragma unroll
            for (int aa = 0; aa < T; ++aa)
#pragma unroll
                for (int cc = 0; cc < T; ++cc)
                    L.gl[(tr + 16 * aa) * NP + tc + 16 * cc] = c[aa][cc];
        }
        const YCoef cur = nxt;
        // the next y-line's coefficients (the last one loads its own again)
        const int an = a + da != a1 ? a + da : a;
        nxt = yf_coef_load(S, ny, an, ab_of(an), Dc, Uc);
        yf_coef_put(cur, S, ab, NP, L.cb, YB);
        __syncthreads();
#pragma unroll
        for (int aa = 0; aa < T; ++aa)
#pragma unroll
            for (int cc = 0; cc < T; ++cc) c[aa][cc] = yf_a(L.cb, NP, n, tr + 16 * aa, tc + 16 * cc);
        if (!first) yf_sandwich(c, L, tr, tc, half);
        yf_invert(c, L, tr, tc);
        yf_store(c, YF + S.yoff + (long)a * nn, n, tr, tc);
    }
}

// The middle line of every strip: C = A_m - B_{m-1}^T T_{m-1}^{-1} B_{m-1}
// - B_m U_{m+1}^{-1} B_m^T (the terms present), inverted.
template <int T, typename E>
__global__ __launch_bounds__(YF_THREADS) void yfactor_mid_kernel(const YStrip *ys, int ny,
                                                                 const double2 *Dc,
                                                                 const double2 *Uc, E *YF,
                                                                 double2 *YB) {
    constexpr int NP = 16 * T;
    const YStrip S = ys[blockIdx.x];
    const int n = S.nx, ld = yld<E>(n), nn = n * ld, m = (ny - 1) / 2;
    extern __shared__ double2 ylds[];
    const YFLds<T> L = yf_lds<T>(ylds);
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    yf_init(L);
    __syncthreads();
    double2 c[T][T];
    yf_coef_put(yf_coef_load(S, ny, m, -1, Dc, Uc), S, -1, NP, L.cb, YB);
    __syncthreads();
#pragma unroll
    for (int aa = 0; aa < T; ++aa)
#pragma unroll
        for (int cc = 0; cc < T; ++cc) c[aa][cc] = yf_a(L.cb, NP, n, tr + 16 * aa, tc + 16 * cc);
    __syncthreads();
    for (int side = 0; side < 2; ++side) {
        const int ab = side == 0 ? m - 1 : m;           // coupling block index
        const int ag = side == 0 ? m - 1 : m + 1;       // neighbouring complement
        if (ag < 0 || ag >= ny) continue;
        yf_coef_put(yf_coef_load(S, ny, m, ab, Dc, Uc), S, ab, NP, L.cb, YB);
        const E *src = YF + S.yoff + (long)ag * nn;
        for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {
            const int i = e / NP, k = e % NP;
            L.gl[e] = (i < n && k < n) ? y2d(src[i * ld + k]) : cd(i == k ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
        yf_sandwich(c, L, tr, tc, side);
    }
    yf_invert(c, L, tr, tc);
    yf_store(c, YF + S.yoff + (long)m * nn, n, tr, tc);
}

// Registers of the factor for strips of at most max_nx node-lines: the
// padded order NP = 16 T >= max_nx.
int yf_t(int max_nx) { return max_nx <= 32 ? 2 : (max_nx <= 48 ? 3 : 4); }

// ---------------------------------------------------------------- solve
// One workgroup per strip half covers 8 NR rows, NR = ceil(max nx / 8) (4,
// 6 or 8, a template parameter).  LPR lanes serve a row: 8 with FP64
// storage, 4 with complex FP32 storage (16-byte loads carry two entries
// there), so a wave owns 64 / LPR rows and the workgroup has NR LPR / 8
// waves.  Lane slice qs = lane % LPR of row i holds the entries of the
// inverse G the step multiplies by: FP64, G[q][i] for q = qs + 8 r (G is
// symmetric, so these are row i's terms); FP32, the pairs (G[i][q],
// G[i][q+1]) for q = 2 qs + 8 r; r < NR either way.  It also holds one more
// value of row i: qs 1 the coupling block's diagonal, qs 2 its entry towards
// row i + 1, qs 3 the one towards row i - 1 (for the product with B^T or
// with B), qs YQ_RHS the right-hand side.  A row's sums are formed within
// its lanes by DPP; rows meet in LDS.  The data of the next YS_DEPTH - 1
// steps are loaded while the current one computes.  Halving the waves with
// FP32 storage halves the instructions the busiest SIMD issues per step (a
// step is a few hundred instructions of dependent arithmetic, group sums and
// LDS traffic between two barriers).
constexpr int YS_DEPTH = 4;
template <typename E>
__host__ __device__ constexpr int ylpr() { return sizeof(E) == 8 ? 4 : 8; }
template <typename E>
__host__ __device__ constexpr int yq_rhs() { return sizeof(E) == 8 ? 0 : 6; }
template <int NR, typename E>
__host__ __device__ constexpr int ywaves() { return NR * ylpr<E>() / 8; }

template <int NR, typename E>
struct YStage {
    typename std::conditional<sizeof(E) == 16, double2, float4>::type g[NR];
    double2 ex;     // this lane's coefficient or right-hand-side value
};

// Sum over the LPR lanes of a row group (quad swaps, then for 8 lanes the
// half-row mirror), in every lane of the group.  Every lane of the wave must
// be active.
// (Every source lane of these patterns is valid, so the moves need no old
// value: no register is zeroed before each.)
template <int CTRL>
__device__ __forceinline__ double ydpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int LPR>
__device__ __forceinline__ double ys_gsum(double v) {
    v += ydpp<0xB1>(v);     // quad_perm [1,0,3,2]
    v += ydpp<0x4E>(v);     // quad_perm [2,3,0,1]
    if constexpr (LPR == 8) v += ydpp<0x141>(v);    // row_half_mirror
    return v;
}
template <int LPR>
__device__ __forceinline__ double2 ys_gsum2(double2 v) {
    return cd(ys_gsum<LPR>(v.x), ys_gsum<LPR>(v.y));
}

// Buffer resource over one inverse (n^2 complex values): a lane whose
// offset lies past it reads zeros without a memory request.  The base and
// size are the same in every lane (scalar registers).
template <typename E>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t ys_block(const E *G, int nn) {
    const unsigned long long b = reinterpret_cast<unsigned long long>(G);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    void *p = reinterpret_cast<void *>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0,
                                             __builtin_amdgcn_readfirstlane(nn * (int)sizeof(E)),
                                             0x00020000);
}

// Loads of one step, all unconditional (a load under a branch would make
// the compiler wait for every load in flight): G[q][i] through the block's
// resource, lanes with q >= n or i >= n reading zeros; the lane's extra
// value from an index clamped into its array (rows i >= n are never
// stored).  yb: the step's coupling block (y-line-major), tr = 1 for the
// product with B, 0 for B^T; src: the right-hand side's packed lines.
template <int NR, typename E>
__device__ __forceinline__ void ys_load(YStage<NR, E> &s, const E *G, const double2 *yb,
                                        const double2 *src, long off, int ny, int a, int n, int i,
                                        int qs, int tr) {
    const int ic = min(i, n - 1), im = max(ic - 1, 0);
    const int ld = yld<E>(n);
    const __amdgpu_buffer_rsrc_t rs = ys_block(G, n * ld);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        unsigned bo;
        if constexpr (sizeof(E) == 16) {
            const int q = qs + 8 * r;
            bo = (q < n && i < n) ? (unsigned)(q * n + i) * 16u : 0xFFFFFFF0u;
        } else {   // q even and ld even: the pair lies within row i
            const int q = 2 * qs + 8 * r;
            bo = (q < ld && i < n) ? (unsigned)(i * ld + q) * 8u : 0xFFFFFFF0u;
        }
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, bo, 0, 0);
        __builtin_memcpy(&s.g[r], &v, 16);
    }
    // (B t)_i = B[i][i] t_i + B[i][i+1] t_{i+1} + B[i][i-1] t_{i-1} and
    // (B^T t)_i = B[i][i] t_i + B[i+1][i] t_{i+1} + B[i-1][i] t_{i-1}, with
    // B[l][l+1] at yb[n + l] and B[l+1][l] at yb[2n + l]
    const int ci = qs == 2 ? (tr ? n : 2 * n) + ic : (qs == 3 ? (tr ? 2 * n : n) + im : ic);
    const double2 *p = qs == yq_rhs<E>() ? src + (off + ic) * ny + a : yb + ci;
    s.ex = *p;
}

// This lane's product over its q slice: sum_r G[q][i] v[q].
template <int NR, typename E>
__device__ __forceinline__ double2 ys_partial(const YStage<NR, E> &s, const double2 *v, int qs) {
    double2 a0 = yz(), a1 = yz();
    if constexpr (sizeof(E) == 16) {
#pragma unroll
        for (int r = 0; r < NR; r += 2) {
            a0 = yfma(s.g[r], v[qs + 8 * r], a0);
            a1 = yfma(s.g[r + 1], v[qs + 8 * (r + 1)], a1);
        }
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int q = 2 * qs + 8 * r;
            a0 = yfma(cd((double)s.g[r].x, (double)s.g[r].y), v[q], a0);
            a1 = yfma(cd((double)s.g[r].z, (double)s.g[r].w), v[q + 1], a1);
        }
    }
    return cd(a0.x + a1.x, a0.y + a1.y);
}

// rhs - (coupling product)_i from the row's lanes; tl holds the product's
// input vector at tl[1 + j] (tl[0] = 0 for j = -1).  with_rhs = 0 leaves
// the right-hand side out.
template <int NR, typename E>
__device__ __forceinline__ double2 ys_couple(const YStage<NR, E> &s, const double2 *tl, int i, int qs,
                                            bool with_rhs) {
    const int j = qs == 2 ? i + 1 : (qs == 3 ? i - 1 : i);
    const double2 t = tl[1 + min(j, 63)];
    const bool c = qs == 1 || qs == 2 || (qs == 3 && i > 0);
    const double2 m = ymul(ysel(c, s.ex, yz()), t);
    const double2 own = ysel(qs == yq_rhs<E>() && with_rhs, s.ex, yz());
    return ys_gsum2<ylpr<E>()>(cd(own.x - m.x, own.y - m.y));
}

// L2 prefetch.  A chain's y-lines are read once, in order, from HBM, and
// only half the CUs run chains, so each chain is bound by the loads one CU
// keeps in flight.  Every chain therefore has a helper workgroup on the
// same XCD (workgroups are dealt to the XCDs round-robin, so helper
// h0 + c of chain c, h0 a multiple of 8, shares its L2) that reads the
// inverses and coupling coefficients of the chain's next YP_LEAD steps into
// L2, paced by the chain's progress word: (epoch << 20) + steps done,
// written by every lane of the chain after each step.  Wave 0 of the helper
// only paces (a bounded wait of YP_SPINS sleeps; after one that runs out
// the helper stops pacing for the sweep, which costs cache space, not
// correctness) and releases the
// others at a barrier; waves 1..7 only load, into a ring of 4 steps whose
// values are summed 2 steps later, so neither waits on the other's memory
// operations.
constexpr int YP_LEAD = 8;
constexpr unsigned YP_SPINS = 1u << 14;

// loads per loading thread and step: one per 128-byte line of an inverse
// ((8 NR)^2 entries of es bytes) over the 64 (nw - 1) loading threads, and
// one coupling coefficient
constexpr int yp_q(int nr, int nw, int es) {
    return ((64 * nr * nr * es + 127) / 128 + 64 * (nw - 1) - 1) / (64 * (nw - 1)) + 1;
}

template <bool FWD, int NR, typename E>
__device__ void ys_helper(const YStrip &S, int ny, int half, const E *YF,
                          const double2 *YB, unsigned long long *prog, unsigned long long base) {
    constexpr int NW = ywaves<NR, E>(), YP_Q = yp_q(NR, NW, (int)sizeof(E)), NL = 64 * (NW - 1);
    constexpr int EPL = 128 / (int)sizeof(E);   // entries per line
    const int n = S.nx, nn = n * yld<E>(n), m = (ny - 1) / 2;
    const int a0 = FWD ? (half == 0 ? 0 : ny - 1) : (half == 0 ? m - 1 : m + 1);
    const int da = FWD ? (half == 0 ? 1 : -1) : (half == 0 ? -1 : 1);
    const int steps = half == 0 ? m : ny - 1 - m;
    const int wave = threadIdx.x >> 6, lt = (int)threadIdx.x - 64;   // loader index
    double acc = 0.0;
    double ring[4][YP_Q];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < YP_Q; ++q) ring[u][q] = 0.0;
    auto touch = [&](double (&r)[YP_Q], int k) {
        const int a = a0 + min(k, steps - 1) * da;
        const int ag = FWD ? (k > 0 ? a - da : a) : a;
        const int ab = max(FWD ? (half == 0 ? a - 1 : a) : (half == 0 ? a : a - 1), 0);
        const E *G = YF + S.yoff + (long)ag * nn;
#pragma unroll
        for (int q = 0; q < YP_Q - 1; ++q) r[q] = (double)G[min((lt + NL * q) * EPL, nn - 1)].x;
        r[YP_Q - 1] = YB[S.boff + (long)ab * 3 * n + min(lt * 8, 3 * n - 1)].x;
    };
    auto fold = [&](const double (&r)[YP_Q]) {
#pragma unroll
        for (int q = 0; q < YP_Q; ++q) acc += r[q];
    };
    // the pacer and the loaders pass one barrier per step each
    if (wave == 0) {
        bool pace = true;   // off for the rest of the sweep after one timed-out wait
        for (int k = 0; k < steps; ++k) {
            if (threadIdx.x == 0 && pace && k >= YP_LEAD) {
                unsigned spins = 0;
                while (__hip_atomic_load(prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       base + (unsigned long long)(k - YP_LEAD)) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins >= YP_SPINS) {
                        pace = false;
                        break;
                    }
                }
            }
            __syncthreads();
        }
        return;
    }
    for (int k0 = 0; k0 < steps; k0 += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u;
            if (k >= steps) break;
            touch(ring[u], k);
            __syncthreads();
            fold(ring[(u + 2) & 3]);   // the step 2 back, summed after this step's loads
        }
    }
    // keeps the loads: the sum is never this value
    if (acc == -1.0e300) prog[0] = 0;
}

// Forward sweeps, blockIdx.x = 2 j + half: lower w_a = b_a - B_{a-1}^T
// T_{a-1}^{-1} w_{a-1} for a = 0 .. m - 1, upper v_a = b_a - B_a U_{a+1}^{-1}
// v_{a+1} for a = ny - 1 .. m + 1; w and v are written over x.  Step k
// (a = a0 + k da) multiplies by the inverse of y-line a - da and coupling
// block a - 1 (lower, B^T) or a (upper, B).
template <int NR, typename E>
__global__ __launch_bounds__((64 * ywaves<NR, E>())) void ysolve_fwd_kernel(
    const YStrip *ys, int ny, const E *YF, const double2 *YB, const double2 *b, double2 *x,
    const StepCtl *c, int *ran, int nchain, unsigned long long *prog, unsigned long long epoch) {
    if (yidle(c)) return;
    const int h0 = (nchain + 7) & ~7;
    const unsigned long long base = epoch << 20;
    if ((int)blockIdx.x >= nchain) {
        const int ch = (int)blockIdx.x - h0;
        if (ch >= 0 && ch < nchain)
            ys_helper<true, NR, E>(ys[ch >> 1], ny, ch & 1, YF, YB, prog + ch, base);
        return;
    }
    if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
    unsigned long long *my = prog + blockIdx.x;
    const int j = blockIdx.x >> 1, half = blockIdx.x & 1;
    const YStrip S = ys[j];
    const int n = S.nx, nn = n * yld<E>(n), m = (ny - 1) / 2;
    constexpr int LPR = ylpr<E>();
    const int lane = threadIdx.x & 63, i = (threadIdx.x >> 6) * (64 / LPR) + lane / LPR;
    const int qs = lane % LPR;
    __shared__ double2 v[64], tl[66];
    const int a0 = half == 0 ? 0 : ny - 1, da = half == 0 ? 1 : -1;
    const int steps = half == 0 ? m : ny - 1 - m;
    const int tr = half;
    if (threadIdx.x < 64) v[threadIdx.x] = yz();
    if (threadIdx.x < 66) tl[threadIdx.x] = yz();
    // step k's data; steps past the end reload the last one (unused), step
    // 0 has no product and points G and yb at y-line 0's (unused)
    auto load = [&](YStage<NR, E> &st, int k) {
        k = min(k, steps - 1);
        const int a = a0 + k * da;
        const int ag = k > 0 ? a - da : 0, ab = k > 0 ? (half == 0 ? a - 1 : a) : 0;
        ys_load(st, YF + S.yoff + (long)ag * nn, YB + S.boff + (long)ab * 3 * n, b, S.off, ny,
                a, n, i, qs, tr);
    };
    auto step = [&](const YStage<NR, E> &st, int k) {
        const int a = a0 + k * da;
        if (k > 0) {
            const double2 t = ys_gsum2<LPR>(ys_partial(st, v, qs));
            if (qs == 0 && i < n) tl[1 + i] = t;
            __syncthreads();
        }
        const double2 val = ys_couple(st, tl, i, qs, true);
        if (qs == 0 && i < n) {
            v[i] = val;
            x[(long)(S.off + i) * ny + a] = val;
        }
        *my = base + (unsigned long long)(k + 1);   // progress, for the helper
        __syncthreads();
    };
    YStage<NR, E> s0, s1, s2, s3;
    load(s0, 0);
    load(s1, 1);
    load(s2, 2);
    __syncthreads();
    for (int k = 0; k < steps; k += YS_DEPTH) {
        load(s3, k + 3);
        step(s0, k);
        if (k + 1 >= steps) break;
        load(s0, k + 4);
        step(s1, k + 1);
        if (k + 2 >= steps) break;
        load(s1, k + 5);
        step(s2, k + 2);
        if (k + 3 >= steps) break;
        load(s2, k + 6);
        step(s3, k + 3);
    }
}

// Backward sweeps: lower x_a = T_a^{-1}(w_a - B_a x_{a+1}) for a = m - 1
// down to 0, upper x_a = U_a^{-1}(v_a - B_{a-1}^T x_{a-1}) for a = m + 1 up.
// Step k (a = a0 + k da) multiplies by the inverse of y-line a, coupling
// block a (lower, B) or a - 1 (upper, B^T), and reads w_a / v_a from x.
template <int NR, typename E>
__global__ __launch_bounds__((64 * ywaves<NR, E>())) void ysolve_bwd_kernel(
    const YStrip *ys, int ny, const E *YF, const double2 *YB, double2 *x, const StepCtl *c,
    int nchain, unsigned long long *prog, unsigned long long epoch) {
    if (yidle(c)) return;
    const int h0 = (nchain + 7) & ~7;
    const unsigned long long base = epoch << 20;
    if ((int)blockIdx.x >= nchain) {
        const int ch = (int)blockIdx.x - h0;
        if (ch >= 0 && ch < nchain)
            ys_helper<false, NR, E>(ys[ch >> 1], ny, ch & 1, YF, YB, prog + ch, base);
        return;
    }
    unsigned long long *my = prog + blockIdx.x;
    const int j = blockIdx.x >> 1, half = blockIdx.x & 1;
    const YStrip S = ys[j];
    const int n = S.nx, nn = n * yld<E>(n), m = (ny - 1) / 2;
    constexpr int LPR = ylpr<E>();
    const int lane = threadIdx.x & 63, i = (threadIdx.x >> 6) * (64 / LPR) + lane / LPR;
    const int qs = lane % LPR;
    __shared__ double2 v[64], tl[66];
    const int a0 = half == 0 ? m - 1 : m + 1, da = half == 0 ? -1 : 1;
    const int steps = half == 0 ? m : ny - 1 - m;
    const int tr = half == 0 ? 1 : 0;
    if (threadIdx.x < 64) v[threadIdx.x] = yz();
    if (threadIdx.x < 66) tl[threadIdx.x] = yz();
    __syncthreads();
    // x_m, the start of both sweeps
    if (qs == 0 && i < n) tl[1 + i] = x[(long)(S.off + i) * ny + m];
    __syncthreads();
    auto load = [&](YStage<NR, E> &st, int k) {
        k = min(k, steps - 1);   // past the end: the last step's data again (unused)
        const int a = a0 + k * da;
        const int ab = half == 0 ? a : a - 1;
        ys_load(st, YF + S.yoff + (long)a * nn, YB + S.boff + (long)ab * 3 * n, x, S.off, ny, a,
                n, i, qs, tr);
    };
    auto step = [&](const YStage<NR, E> &st, int k) {
        const int a = a0 + k * da;
        const double2 r = ys_couple(st, tl, i, qs, true);
        if (qs == 0 && i < n) v[i] = r;
        __syncthreads();
        const double2 t = ys_gsum2<LPR>(ys_partial(st, v, qs));
        if (qs == 0 && i < n) {
            tl[1 + i] = t;
            x[(long)(S.off + i) * ny + a] = t;
        }
        *my = base + (unsigned long long)(k + 1);   // progress, for the helper
        __syncthreads();
    };
    YStage<NR, E> s0, s1, s2, s3;
    load(s0, 0);
    load(s1, 1);
    load(s2, 2);
    for (int k = 0; k < steps; k += YS_DEPTH) {
        load(s3, k + 3);
        step(s0, k);
        if (k + 1 >= steps) break;
        load(s0, k + 4);
        step(s1, k + 1);
        if (k + 2 >= steps) break;
        load(s1, k + 5);
        step(s2, k + 2);
        if (k + 3 >= steps) break;
        load(s2, k + 6);
        step(s3, k + 3);
    }
}

// Middle line: x_m = M_m^{-1}(b_m - B_{m-1}^T T_{m-1}^{-1} w_{m-1} - B_m
// U_{m+1}^{-1} v_{m+1}), the terms present; three products of one step
// each, all their data loaded up front.
template <int NR, typename E>
__global__ __launch_bounds__((64 * ywaves<NR, E>())) void ysolve_mid_kernel(const YStrip *ys, int ny,
                                                                const E *YF,
                                                                const double2 *YB,
                                                                const double2 *b, double2 *x,
                                                                const StepCtl *c) {
    if (yidle(c)) return;
    const YStrip S = ys[blockIdx.x];
    const int n = S.nx, nn = n * yld<E>(n), m = (ny - 1) / 2;
    constexpr int LPR = ylpr<E>();
    const int lane = threadIdx.x & 63, i = (threadIdx.x >> 6) * (64 / LPR) + lane / LPR;
    const int qs = lane % LPR;
    __shared__ double2 v[64], tl[66];
    if (threadIdx.x < 64) v[threadIdx.x] = yz();   // entries q >= n meet clamped G values
    if (threadIdx.x < 66) tl[threadIdx.x] = yz();
    const bool lo = m - 1 >= 0, hi = m + 1 < ny;
    YStage<NR, E> sl, sh, sm;
    // lower side: inverse of m - 1, coupling block m - 1 (B^T), w_{m-1} from
    // x; upper side: inverse of m + 1, coupling block m (B), v_{m+1} from x
    // (a missing side points at y-line m's data, unused); the middle
    // product: inverse of m, b_m (coupling entries of block 0, unused)
    const int al = lo ? m - 1 : m, ah = hi ? m + 1 : m, bl = lo ? m - 1 : 0, bh = hi ? m : 0;
    ys_load(sl, YF + S.yoff + (long)al * nn, YB + S.boff + (long)bl * 3 * n, x, S.off, ny, al,
            n, i, qs, 0);
    ys_load(sh, YF + S.yoff + (long)ah * nn, YB + S.boff + (long)bh * 3 * n, x, S.off, ny, ah,
            n, i, qs, 1);
    ys_load(sm, YF + S.yoff + (long)m * nn, YB + S.boff, b, S.off, ny, m, n, i, qs, 0);
    __syncthreads();
    double2 acc = yz();
    auto side = [&](const YStage<NR, E> &st) {
        // the side's vector (the right-hand-side slot of its stage) into v
        if (qs == yq_rhs<E>() && i < n) v[i] = st.ex;
        __syncthreads();
        const double2 t = ys_gsum2<LPR>(ys_partial(st, v, qs));
        if (qs == 0 && i < n) tl[1 + i] = t;
        __syncthreads();
        const double2 cpl = ys_couple(st, tl, i, qs, false);   // -(coupling product)_i
        acc.x += cpl.x;
        acc.y += cpl.y;
        __syncthreads();
    };
    if (lo) side(sl);
    if (hi) side(sh);
    // b_m from the middle stage's right-hand-side lane, to the whole row
    const double2 rb = ys_gsum2<LPR>(ysel(qs == yq_rhs<E>(), sm.ex, yz()));
    if (qs == 0 && i < n) v[i] = cd(rb.x + acc.x, rb.y + acc.y);
    __syncthreads();
    const double2 t = ys_gsum2<LPR>(ys_partial(sm, v, qs));
    if (qs == 0 && i < n) x[(long)(S.off + i) * ny + m] = t;
}

}  // namespace

size_t yorder_factor_lds(int max_nx) {
    return sizeof(double2) * (size_t)yf_lds_count(16 * yf_t(max_nx));
}

// Per y-line: the inversion (n^3 complex multiply-adds) and the two
// products with the tridiagonal coupling block (6 n^2), 8 real flops each.
double yorder_factor_flops(int ny, int nx) {
    const double n = nx;
    return (double)ny * 8.0 * (n * n * n + 6.0 * n * n);
}

template <typename E>
static hipError_t yfactor_typed(hipStream_t st, const YStrip *ys, int nstrips, int ny, int max_nx,
                                const double2 *Dc, const double2 *Uc, E *YF, double2 *YB) {
    const size_t lds = yorder_factor_lds(max_nx);
    auto go = [&](auto half, auto mid) {
        hipLaunchKernelGGL(half, dim3(2 * nstrips), dim3(YF_THREADS), lds, st, ys, ny, Dc, Uc, YF,
                           YB);
        hipLaunchKernelGGL(mid, dim3(nstrips), dim3(YF_THREADS), lds, st, ys, ny, Dc, Uc, YF, YB);
    };
    if (max_nx <= 32) go(yfactor_half_kernel<2, E>, yfactor_mid_kernel<2, E>);
    else if (max_nx <= 48) go(yfactor_half_kernel<3, E>, yfactor_mid_kernel<3, E>);
    else if (max_nx <= 64) go(yfactor_half_kernel<4, E>, yfactor_mid_kernel<4, E>);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_yfactor(hipStream_t st, const YStrip *ys, int nstrips, int ny, int max_nx,
                          const double2 *Dc, const double2 *Uc, void *YF, int fp32, double2 *YB,
                          hipEvent_t ev0, hipEvent_t ev1) {
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    e = fp32 ? yfactor_typed(st, ys, nstrips, ny, max_nx, Dc, Uc, (float2 *)YF, YB)
             : yfactor_typed(st, ys, nstrips, ny, max_nx, Dc, Uc, (double2 *)YF, YB);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, st);
    return e;
}

template <typename E>
static hipError_t ysolve_typed(hipStream_t st, const YStrip *ys, int nstrips, int ny, int max_nx,
                               const E *YF, const double2 *YB, const double2 *b, double2 *x,
                               const StepCtl *c, int *ran, unsigned long long *prog,
                               unsigned long long ef, unsigned long long eb) {
    // chains 0 .. 2N-1, then (from the next multiple of 8) their helpers
    const int nchain = 2 * nstrips, grid = ((nchain + 7) & ~7) + nchain;
    auto go = [&](auto fwd, auto mid, auto bwd, int nr) {
        const dim3 block((unsigned)(8 * nr * ylpr<E>()));   // 64 NR LPR / 8 threads
        hipLaunchKernelGGL(fwd, dim3(grid), block, 0, st, ys, ny, YF, YB, b, x, c, ran, nchain,
                           prog, ef);
        hipLaunchKernelGGL(mid, dim3(nstrips), block, 0, st, ys, ny, YF, YB, b, x, c);
        hipLaunchKernelGGL(bwd, dim3(grid), block, 0, st, ys, ny, YF, YB, x, c, nchain, prog,
                           eb);
    };
    if (max_nx <= 32)
        go(ysolve_fwd_kernel<4, E>, ysolve_mid_kernel<4, E>, ysolve_bwd_kernel<4, E>, 4);
    else if (max_nx <= 48)
        go(ysolve_fwd_kernel<6, E>, ysolve_mid_kernel<6, E>, ysolve_bwd_kernel<6, E>, 6);
    else if (max_nx <= 64)
        go(ysolve_fwd_kernel<8, E>, ysolve_mid_kernel<8, E>, ysolve_bwd_kernel<8, E>, 8);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ysolve(hipStream_t st, const YStrip *ys, int nstrips, int ny, int max_nx,
                         const void *YF, int fp32, const double2 *YB, const double2 *b,
                         double2 *x, const StepCtl *c, int *ran, unsigned long long *prog,
                         unsigned long long *epoch, hipEvent_t ev0, hipEvent_t ev1) {
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    const unsigned long long ef = ++*epoch, eb = ++*epoch;
    e = fp32 ? ysolve_typed(st, ys, nstrips, ny, max_nx, (const float2 *)YF, YB, b, x, c, ran,
                            prog, ef, eb)
             : ysolve_typed(st, ys, nstrips, ny, max_nx, (const double2 *)YF, YB, b, x, c, ran,
                            prog, ef, eb);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, st);
    return e;
}
