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
// factor is the inverse of every complement (nx x nx, FP64), nx^2 per y-line
// instead of the ny^2 per node-line of the node-line order.  The
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
// c ? a : b, component-wise (a conditional on the struct itself selects
// between addresses and keeps the values out of registers)
__device__ __forceinline__ double2 ysel(bool c, double2 a, double2 b) {
    return cd(c ? a.x : b.x, c ? a.y : b.y);
}

// ---------------------------------------------------------------- factor
// A workgroup of 256 threads per strip half: thread (k = tid mod n, rg = tid
// div n) owns column k of rows rg + ng r, r < R (ng = 256 div n row groups;
// R >= ceil(n / ng), a template parameter); threads with rg >= ng idle.
// Rows i >= n of a thread are computed on clamped data and never published
// or stored.
constexpr int YF_THREADS = 256;
constexpr int YF_COLB = 65;    // pivot column buffer: rows < n <= 64, and a slot that
                               // takes the writes of rows >= n (never read)

// LDS of a factor workgroup: the pivot row (2 x 64) and column (2 x 65) of
// the current and the next pivot, A's two diagonals and the coupling block's
// three (5 n), the previous inverse and then the product H (n^2).
struct YFactorLds {
    double2 *cb, *gl, *rowb, *colb;
};
__device__ __forceinline__ YFactorLds yf_lds(double2 *base, int n) {
    YFactorLds L;
    L.rowb = base;                                // 2 x 64
    L.colb = base + 128;                          // 2 x YF_COLB
    L.cb = base + 128 + 2 * YF_COLB;              // 5 n
    L.gl = base + 128 + 2 * YF_COLB + 5 * n;      // n^2
    return L;
}

// Coefficients of y-line a: A's diagonal and off-diagonal (cb[0, 2n)) and,
// when ab >= 0, the coupling block B_ab's diagonal, upper and lower entries
// (cb[2n, 5n)), also written y-line-major to YB for the solve.
__device__ void yf_coef(const YStrip &S, int ny, int a, int ab, const double2 *Dc,
                        const double2 *Uc, double2 *cb, double2 *YB) {
    const int n = S.nx;
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
        const long r = ((long)(S.off + l) * ny + a) * 3;
        cb[l] = Dc[r + 1];
        cb[n + l] = l + 1 < n ? Uc[r + 1] : yz();
        if (ab >= 0) {
            const long rb = ((long)(S.off + l) * ny + ab) * 3;
            const double2 d = Dc[rb + 2];
            const double2 up = l + 1 < n ? Uc[rb + 2] : yz();
            const double2 lo = l + 1 < n ? Uc[((long)(S.off + l) * ny + ab + 1) * 3 + 0] : yz();
            cb[2 * n + l] = d;
            cb[3 * n + l] = up;
            cb[4 * n + l] = lo;
            double2 *yb = YB + S.boff + (long)ab * 3 * n;
            yb[l] = d;
            yb[n + l] = up;
            yb[2 * n + l] = lo;
        }
    }
}

// The coefficients one thread (row l = min(tid, n - 1)) contributes to
// y-line a's LDS copy: A's diagonal and off-diagonal, and B_ab's diagonal,
// upper and lower entries.  Loaded unconditionally (ab clamped to 0 when
// there is no coupling block) so that the next y-line's loads can be in
// flight while the current one is inverted; put() applies the masks.
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
__device__ __forceinline__ void yf_coef_put(const YCoef &q, const YStrip &S, int ab, double2 *cb,
                                            double2 *YB) {
    const int n = S.nx, l = threadIdx.x;
    if (l >= n) return;
    const bool in = l + 1 < n;
    cb[l] = q.ad;
    cb[n + l] = ysel(in, q.ao, yz());
    if (ab >= 0) {
        const double2 up = ysel(in, q.bu, yz()), lo = ysel(in, q.bl, yz());
        cb[2 * n + l] = q.bd;
        cb[3 * n + l] = up;
        cb[4 * n + l] = lo;
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
__device__ __forceinline__ Tri yf_tri(const double2 *cb, int n, int j, int tr) {
    Tri t;
    const double2 *up = cb + 3 * n, *lo = cb + 4 * n;
    const int jm = max(j - 1, 0);
    t.z0 = cb[2 * n + j];
    t.m1 = ysel(j > 0, ysel(tr, lo[jm], up[jm]), yz());
    t.p1 = ysel(j + 1 < n, ysel(tr, up[j], lo[j]), yz());
    return t;
}

// c[r] -= (X G Y)[i_r][k] with G in L.gl (n x n): lower C -= B^T G B, upper
// C -= B G B^T, as H = G Y (3 terms) then X H (3 terms); reads clamped into
// the block (their coefficient is zero where clamping changed the index).
// Ends with L.gl free.
template <int R>
__device__ __forceinline__ void yf_sandwich(double2 (&c)[R], const YFactorLds &L, int n, int k, int rg, int ng,
                            bool act, int tr) {
    double2 h[R];
    const Tri tk = yf_tri(L.cb, n, k, tr);
    const int km = max(k - 1, 0), kp = min(k + 1, n - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double2 *gi = L.gl + min(rg + ng * r, n - 1) * n;
        h[r] = yfma(gi[kp], tk.p1, yfma(gi[km], tk.m1, ymul(gi[k], tk.z0)));
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = rg + ng * r;
        if (act && i < n) L.gl[i * n + k] = h[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = min(rg + ng * r, n - 1);
        const Tri ti = yf_tri(L.cb, n, i, tr);
        const double2 s = yfma(ti.p1, L.gl[min(i + 1, n - 1) * n + k],
                               yfma(ti.m1, L.gl[max(i - 1, 0) * n + k],
                                    ymul(ti.z0, L.gl[i * n + k])));
        c[r].x -= s.x;
        c[r].y -= s.y;
    }
    __syncthreads();
}

// In-place Gauss-Jordan inversion of the complement held in registers,
// without pivoting.  Pivot p reads row p and column p of the current matrix
// from LDS (buffer p & 1) and publishes row and column p + 1 after its
// update into the other buffer: one barrier per pivot.  The pivots run in
// blocks RB of ng (a compile-time block index, so that the register holding
// row p + 1, row group (p + 1) mod ng, slot (p + 1) div ng, is static).
template <int R, int RB>
__device__ __forceinline__ void yf_pivot_block(double2 (&c)[R], const YFactorLds &L, int n,
                                               int k, int rg, int ng, bool act) {
    for (int s = 0; s < ng; ++s) {
        const int p = RB * ng + s;
        if (p >= n) return;
        const int b = p & 1, nb = b ^ 1;
        const double2 *rowp = L.rowb + 64 * b, *colp = L.colb + YF_COLB * b;
        const double2 piv = rowp[p];
        const double inv = 1.0 / (piv.x * piv.x + piv.y * piv.y);
        const double2 d = cd(piv.x * inv, -piv.y * inv);   // 1 / C[p][p]
        // every entry becomes s v - C[i][p] mu and row p becomes mu, with
        // mu = C[p][k] / C[p][p], s = 1 off column p, and mu = 1 / C[p][p],
        // s = 0 on it (where C[i][p] is v itself)
        const bool kpiv = k == p;
        const double2 mu = ysel(kpiv, d, ymul(rowp[k], d));
        const double sv = kpiv ? 0.0 : 1.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double2 v = c[r];
            const double2 f = colp[min(rg + ng * r, n - 1)];
            const double2 nv = cd(fma(sv, v.x, fma(f.y, mu.y, -f.x * mu.x)),
                                  fma(sv, v.y, -fma(f.x, mu.y, f.y * mu.x)));
            // row p = RB ng + s is slot RB of row group s
            c[r] = r == RB ? ysel(rg == s, mu, nv) : nv;
        }
        if (p + 1 < n && act) {
            // row p + 1: row group s + 1 (slot RB), or row group 0 (slot
            // RB + 1) when s + 1 == ng
            const bool wrap = s + 1 == ng;
            constexpr int RN = RB + 1 < R ? RB + 1 : RB;
            if (rg == (wrap ? 0 : s + 1)) L.rowb[64 * nb + k] = ysel(wrap, c[RN], c[RB]);
            if (k == p + 1) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = rg + ng * r;
                    L.colb[YF_COLB * nb + (i < n ? i : YF_COLB - 1)] = c[r];
                }
            }
        }
        __syncthreads();
    }
}

template <int R, int... RBs>
__device__ __forceinline__ void yf_pivot_blocks(double2 (&c)[R], const YFactorLds &L, int n,
                                                int k, int rg, int ng, bool act,
                                                std::integer_sequence<int, RBs...>) {
    (yf_pivot_block<R, RBs>(c, L, n, k, rg, ng, act), ...);
}

template <int R>
__device__ __forceinline__ void yf_invert(double2 (&c)[R], const YFactorLds &L, int n, int k, int rg, int ng,
                          bool act) {
    if (act && rg == 0) L.rowb[k] = c[0];
    if (act && k == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (rg + ng * r < n) L.colb[rg + ng * r] = c[r];
    }
    __syncthreads();
    yf_pivot_blocks(c, L, n, k, rg, ng, act, std::make_integer_sequence<int, R>());
}

// A_a[i][k] from cb
__device__ __forceinline__ double2 yf_a(const double2 *cb, int n, int i, int k) {
    const int mn = min(min(i, k), n - 1);
    const double2 dg = cb[min(i, n - 1)], od = cb[n + mn];
    return ysel(i == k, dg, ysel(k == i + 1 || i == k + 1, od, yz()));
}

template <int R>
__device__ __forceinline__ void yf_store(const double2 (&c)[R], double2 *out, int n, int k,
                                         int rg, int ng, bool act) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = rg + ng * r;
        if (act && i < n) out[i * n + k] = c[r];
    }
}

// The two halves of every strip: blockIdx.x = 2 j + half.
template <int R>
__global__ __launch_bounds__(YF_THREADS) void yfactor_half_kernel(const YStrip *ys, int ny,
                                                                  const double2 *Dc,
                                                                  const double2 *Uc, double2 *YF,
                                                                  double2 *YB) {
    const int j = blockIdx.x >> 1, half = blockIdx.x & 1;
    const YStrip S = ys[j];
    const int n = S.nx, nn = n * n, m = (ny - 1) / 2;
    extern __shared__ double2 ylds[];
    const YFactorLds L = yf_lds(ylds, n);
    const int ng = YF_THREADS / n, k = threadIdx.x % n, rg = threadIdx.x / n;
    const bool act = rg < ng;
    double2 c[R];
    const int a0 = half == 0 ? 0 : ny - 1, a1 = m, da = half == 0 ? 1 : -1;
    // coupling block of y-line a: lower B_{a-1}, upper B_a (none for a0)
    auto ab_of = [&](int a) { return a == a0 ? -1 : (half == 0 ? a - 1 : a); };
    YCoef nxt = yf_coef_load(S, ny, a0, -1, Dc, Uc);
    for (int a = a0; a != a1; a += da) {
        const bool first = a == a0;
        const int ab = ab_of(a);
        if (!first) yf_store(c, L.gl, n, k, rg, ng, act);   // the previous inverse
        const YCoef cur = nxt;
        // the next y-line's coefficients (the last one loads its own again)
        const int an = a + da != a1 ? a + da : a;
        nxt = yf_coef_load(S, ny, an, ab_of(an), Dc, Uc);
        yf_coef_put(cur, S, ab, L.cb, YB);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) c[r] = yf_a(L.cb, n, rg + ng * r, k);
        if (!first) yf_sandwich(c, L, n, k, rg, ng, act, half);
        yf_invert(c, L, n, k, rg, ng, act);
        yf_store(c, YF + S.yoff + (long)a * nn, n, k, rg, ng, act);
    }
}

// The middle line of every strip: C = A_m - B_{m-1}^T T_{m-1}^{-1} B_{m-1}
// - B_m U_{m+1}^{-1} B_m^T (the terms present), inverted.
template <int R>
__global__ __launch_bounds__(YF_THREADS) void yfactor_mid_kernel(const YStrip *ys, int ny,
                                                                 const double2 *Dc,
                                                                 const double2 *Uc, double2 *YF,
                                                                 double2 *YB) {
    const YStrip S = ys[blockIdx.x];
    const int n = S.nx, nn = n * n, m = (ny - 1) / 2;
    extern __shared__ double2 ylds[];
    const YFactorLds L = yf_lds(ylds, n);
    const int ng = YF_THREADS / n, k = threadIdx.x % n, rg = threadIdx.x / n;
    const bool act = rg < ng;
    double2 c[R];
    yf_coef(S, ny, m, -1, Dc, Uc, L.cb, YB);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) c[r] = yf_a(L.cb, n, rg + ng * r, k);
    __syncthreads();
    for (int side = 0; side < 2; ++side) {
        const int ab = side == 0 ? m - 1 : m;           // coupling block index
        const int ag = side == 0 ? m - 1 : m + 1;       // neighbouring complement
        if (ag < 0 || ag >= ny) continue;
        yf_coef(S, ny, m, ab, Dc, Uc, L.cb, YB);
        const double2 *src = YF + S.yoff + (long)ag * nn;
        for (int e = threadIdx.x; e < nn; e += blockDim.x) L.gl[e] = src[e];
        __syncthreads();
        yf_sandwich(c, L, n, k, rg, ng, act, side);
    }
    yf_invert(c, L, n, k, rg, ng, act);
    yf_store(c, YF + S.yoff + (long)m * nn, n, k, rg, ng, act);
}

// Rows per thread the factor needs for strips of at most max_nx node-lines
// (the largest ceil(n / (256 div n)) over n <= max_nx).
int yf_rows(int max_nx) {
    int r = 1;
    for (int n = 1; n <= max_nx; ++n) {
        const int ng = YF_THREADS / n;
        r = std::max(r, (n + ng - 1) / ng);
    }
    return r;
}

// ---------------------------------------------------------------- solve
// One workgroup of NR waves per strip half, NR = ceil(max nx / 8) (4, 6 or
// 8, a template parameter).  Wave w owns rows i = 8 w +
// (lane >> 3) of the strip's y-line vectors; the 8 lanes of a row (slice
// qs = lane & 7) hold the entries G[q][i], q = qs + 8 r, r < NR, of the inverse a
// step multiplies by (G is symmetric, so these are row i's terms), and one
// more value of row i each: qs 1 the coupling block's diagonal, qs 2 its
// entry towards row i + 1, qs 3 the one towards row i - 1 (for the
// product with B^T or with B), qs 6 the right-hand side.  A row's sums are
// formed within its 8 lanes by DPP; rows meet in LDS.  The data of the next
// YS_DEPTH - 1 steps are loaded while the current one computes.
constexpr int YS_DEPTH = 4;

template <int NR>
struct YStage {
    double2 g[NR];
    double2 ex;     // this lane's coefficient or right-hand-side value
};

// Sum over the 8 lanes of a row group (quad swaps, then the half-row
// mirror), in every lane of the group.  Every lane of the wave must be active.
__device__ __forceinline__ double ys_gsum(double v) {
    v += dpp_f64<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);     // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);    // row_half_mirror
    return v;
}
__device__ __forceinline__ double2 ys_gsum2(double2 v) { return cd(ys_gsum(v.x), ys_gsum(v.y)); }

// Buffer resource over one inverse (n^2 complex values): a lane whose
// offset lies past it reads zeros without a memory request.  The base and
// size are the same in every lane (scalar registers).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t ys_block(const double2 *G, int nn) {
    const unsigned long long b = reinterpret_cast<unsigned long long>(G);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    void *p = reinterpret_cast<void *>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0,
                                             __builtin_amdgcn_readfirstlane(nn * 16), 0x00020000);
}

// Loads of one step, all unconditional (a load under a branch would make
// the compiler wait for every load in flight): G[q][i] through the block's
// resource, lanes with q >= n or i >= n reading zeros; the lane's extra
// value from an index clamped into its array (rows i >= n are never
// stored).  yb: the step's coupling block (y-line-major), tr = 1 for the
// product with B, 0 for B^T; src: the right-hand side's packed lines.
template <int NR>
__device__ __forceinline__ void ys_load(YStage<NR> &s, const double2 *G, const double2 *yb,
                                        const double2 *src, long off, int ny, int a, int n, int i,
                                        int qs, int tr) {
    const int ic = min(i, n - 1), im = max(ic - 1, 0);
    const __amdgpu_buffer_rsrc_t rs = ys_block(G, n * n);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int q = qs + 8 * r;
        const unsigned bo = (q < n && i < n) ? (unsigned)(q * n + i) * 16u : 0xFFFFFFF0u;
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, bo, 0, 0);
        __builtin_memcpy(&s.g[r], &v, sizeof(double2));
    }
    // (B t)_i = B[i][i] t_i + B[i][i+1] t_{i+1} + B[i][i-1] t_{i-1} and
    // (B^T t)_i = B[i][i] t_i + B[i+1][i] t_{i+1} + B[i-1][i] t_{i-1}, with
    // B[l][l+1] at yb[n + l] and B[l+1][l] at yb[2n + l]
    const int ci = qs == 2 ? (tr ? n : 2 * n) + ic : (qs == 3 ? (tr ? 2 * n : n) + im : ic);
    const double2 *p = qs == 6 ? src + (off + ic) * ny + a : yb + ci;
    s.ex = *p;
}

// This lane's product over its q slice: sum_r G[q][i] v[q].
template <int NR>
__device__ __forceinline__ double2 ys_partial(const YStage<NR> &s, const double2 *v, int qs) {
    double2 a0 = yz(), a1 = yz();
#pragma unroll
    for (int r = 0; r < NR; r += 2) {
        a0 = yfma(s.g[r], v[qs + 8 * r], a0);
        a1 = yfma(s.g[r + 1], v[qs + 8 * (r + 1)], a1);
    }
    return cd(a0.x + a1.x, a0.y + a1.y);
}

// rhs - (coupling product)_i from the row's lanes; tl holds the product's
// input vector at tl[1 + j] (tl[0] = 0 for j = -1).  with_rhs = 0 leaves
// the right-hand side out.
template <int NR>
__device__ __forceinline__ double2 ys_couple(const YStage<NR> &s, const double2 *tl, int i, int qs,
                                            bool with_rhs) {
    const int j = qs == 2 ? i + 1 : (qs == 3 ? i - 1 : i);
    const double2 t = tl[1 + min(j, 63)];
    const bool c = qs == 1 || qs == 2 || (qs == 3 && i > 0);
    const double2 m = ymul(ysel(c, s.ex, yz()), t);
    const double2 own = ysel(qs == 6 && with_rhs, s.ex, yz());
    return ys_gsum2(cd(own.x - m.x, own.y - m.y));
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

// loads per loading thread and step: the (8 NR)^2 entries of an inverse over
// the 64 (NR - 1) loading threads, and one coupling coefficient
constexpr int yp_q(int nr) { return (nr * nr + nr - 2) / (nr - 1) + 1; }

template <bool FWD, int NR>
__device__ void ys_helper(const YStrip &S, int ny, int half, const double2 *YF,
                          const double2 *YB, unsigned long long *prog, unsigned long long base) {
    constexpr int YP_Q = yp_q(NR), NL = 64 * (NR - 1);
    const int n = S.nx, nn = n * n, m = (ny - 1) / 2;
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
        const double2 *G = YF + S.yoff + (long)ag * nn;
#pragma unroll
        for (int q = 0; q < YP_Q - 1; ++q) r[q] = G[min(lt + NL * q, nn - 1)].x;
        r[YP_Q - 1] = YB[S.boff + (long)ab * 3 * n + min(lt, 3 * n - 1)].x;
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
template <int NR>
__global__ __launch_bounds__(64 * NR) void ysolve_fwd_kernel(
    const YStrip *ys, int ny, const double2 *YF, const double2 *YB, const double2 *b, double2 *x,
    const StepCtl *c, int *ran, int nchain, unsigned long long *prog, unsigned long long epoch) {
    if (yidle(c)) return;
    const int h0 = (nchain + 7) & ~7;
    const unsigned long long base = epoch << 20;
    if ((int)blockIdx.x >= nchain) {
        const int ch = (int)blockIdx.x - h0;
        if (ch >= 0 && ch < nchain)
            ys_helper<true, NR>(ys[ch >> 1], ny, ch & 1, YF, YB, prog + ch, base);
        return;
    }
    if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
    unsigned long long *my = prog + blockIdx.x;
    const int j = blockIdx.x >> 1, half = blockIdx.x & 1;
    const YStrip S = ys[j];
    const int n = S.nx, nn = n * n, m = (ny - 1) / 2;
    const int lane = threadIdx.x & 63, i = (threadIdx.x >> 6) * 8 + (lane >> 3), qs = lane & 7;
    __shared__ double2 v[64], tl[66];
    const int a0 = half == 0 ? 0 : ny - 1, da = half == 0 ? 1 : -1;
    const int steps = half == 0 ? m : ny - 1 - m;
    const int tr = half;
    if (threadIdx.x < 64) v[threadIdx.x] = yz();
    if (threadIdx.x < 66) tl[threadIdx.x] = yz();
    // step k's data; steps past the end reload the last one (unused), step
    // 0 has no product and points G and yb at y-line 0's (unused)
    auto load = [&](YStage<NR> &st, int k) {
        k = min(k, steps - 1);
        const int a = a0 + k * da;
        const int ag = k > 0 ? a - da : 0, ab = k > 0 ? (half == 0 ? a - 1 : a) : 0;
        ys_load(st, YF + S.yoff + (long)ag * nn, YB + S.boff + (long)ab * 3 * n, b, S.off, ny,
                a, n, i, qs, tr);
    };
    auto step = [&](const YStage<NR> &st, int k) {
        const int a = a0 + k * da;
        if (k > 0) {
            const double2 t = ys_gsum2(ys_partial(st, v, qs));
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
    YStage<NR> s0, s1, s2, s3;
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
template <int NR>
__global__ __launch_bounds__(64 * NR) void ysolve_bwd_kernel(
    const YStrip *ys, int ny, const double2 *YF, const double2 *YB, double2 *x, const StepCtl *c,
    int nchain, unsigned long long *prog, unsigned long long epoch) {
    if (yidle(c)) return;
    const int h0 = (nchain + 7) & ~7;
    const unsigned long long base = epoch << 20;
    if ((int)blockIdx.x >= nchain) {
        const int ch = (int)blockIdx.x - h0;
        if (ch >= 0 && ch < nchain)
            ys_helper<false, NR>(ys[ch >> 1], ny, ch & 1, YF, YB, prog + ch, base);
        return;
    }
    unsigned long long *my = prog + blockIdx.x;
    const int j = blockIdx.x >> 1, half = blockIdx.x & 1;
    const YStrip S = ys[j];
    const int n = S.nx, nn = n * n, m = (ny - 1) / 2;
    const int lane = threadIdx.x & 63, i = (threadIdx.x >> 6) * 8 + (lane >> 3), qs = lane & 7;
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
    auto load = [&](YStage<NR> &st, int k) {
        k = min(k, steps - 1);   // past the end: the last step's data again (unused)
        const int a = a0 + k * da;
        const int ab = half == 0 ? a : a - 1;
        ys_load(st, YF + S.yoff + (long)a * nn, YB + S.boff + (long)ab * 3 * n, x, S.off, ny, a,
                n, i, qs, tr);
    };
    auto step = [&](const YStage<NR> &st, int k) {
        const int a = a0 + k * da;
        const double2 r = ys_couple(st, tl, i, qs, true);
        if (qs == 0 && i < n) v[i] = r;
        __syncthreads();
        const double2 t = ys_gsum2(ys_partial(st, v, qs));
        if (qs == 0 && i < n) {
            tl[1 + i] = t;
            x[(long)(S.off + i) * ny + a] = t;
        }
        *my = base + (unsigned long long)(k + 1);   // progress, for the helper
        __syncthreads();
    };
    YStage<NR> s0, s1, s2, s3;
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
template <int NR>
__global__ __launch_bounds__(64 * NR) void ysolve_mid_kernel(const YStrip *ys, int ny,
                                                                const double2 *YF,
                                                                const double2 *YB,
                                                                const double2 *b, double2 *x,
                                                                const StepCtl *c) {
    if (yidle(c)) return;
    const YStrip S = ys[blockIdx.x];
    const int n = S.nx, nn = n * n, m = (ny - 1) / 2;
    const int lane = threadIdx.x & 63, i = (threadIdx.x >> 6) * 8 + (lane >> 3), qs = lane & 7;
    __shared__ double2 v[64], tl[66];
    if (threadIdx.x < 64) v[threadIdx.x] = yz();   // entries q >= n meet clamped G values
    if (threadIdx.x < 66) tl[threadIdx.x] = yz();
    const bool lo = m - 1 >= 0, hi = m + 1 < ny;
    YStage<NR> sl, sh, sm;
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
    auto side = [&](const YStage<NR> &st) {
        // the side's vector (the right-hand-side slot of its stage) into v
        if (qs == 6 && i < n) v[i] = st.ex;
        __syncthreads();
        const double2 t = ys_gsum2(ys_partial(st, v, qs));
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
    const double2 rb = ys_gsum2(ysel(qs == 6, sm.ex, yz()));
    if (qs == 0 && i < n) v[i] = cd(rb.x + acc.x, rb.y + acc.y);
    __syncthreads();
    const double2 t = ys_gsum2(ys_partial(sm, v, qs));
    if (qs == 0 && i < n) x[(long)(S.off + i) * ny + m] = t;
}

}  // namespace

size_t yorder_factor_lds(int max_nx) {
    return sizeof(double2) *
           (128 + 2 * (size_t)YF_COLB + 5 * (size_t)max_nx + (size_t)max_nx * max_nx);
}

// Per y-line: the inversion (n^3 complex multiply-adds) and the two
// products with the tridiagonal coupling block (6 n^2), 8 real flops each.
double yorder_factor_flops(int ny, int nx) {
    const double n = nx;
    return (double)ny * 8.0 * (n * n * n + 6.0 * n * n);
}

hipError_t launch_yfactor(hipStream_t st, const YStrip *ys, int nstrips, int ny, int max_nx,
                          const double2 *Dc, const double2 *Uc, double2 *YF, double2 *YB,
                          hipEvent_t ev0, hipEvent_t ev1) {
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    const size_t lds = yorder_factor_lds(max_nx);
    const int rows = yf_rows(max_nx);
    auto go = [&](auto half, auto mid) {
        hipLaunchKernelGGL(half, dim3(2 * nstrips), dim3(YF_THREADS), lds, st, ys, ny, Dc, Uc, YF,
                           YB);
        hipLaunchKernelGGL(mid, dim3(nstrips), dim3(YF_THREADS), lds, st, ys, ny, Dc, Uc, YF, YB);
    };
    if (rows <= 4) go(yfactor_half_kernel<4>, yfactor_mid_kernel<4>);
    else if (rows <= 8) go(yfactor_half_kernel<8>, yfactor_mid_kernel<8>);
    else if (rows <= 16) go(yfactor_half_kernel<16>, yfactor_mid_kernel<16>);
    else return hipErrorInvalidValue;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, st);
    return e;
}

hipError_t launch_ysolve(hipStream_t st, const YStrip *ys, int nstrips, int ny, int max_nx,
                         const double2 *YF, const double2 *YB, const double2 *b, double2 *x,
                         const StepCtl *c, int *ran, unsigned long long *prog,
                         unsigned long long *epoch, hipEvent_t ev0, hipEvent_t ev1) {
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    // chains 0 .. 2N-1, then (from the next multiple of 8) their helpers
    const int nchain = 2 * nstrips, grid = ((nchain + 7) & ~7) + nchain;
    const unsigned long long ef = ++*epoch, eb = ++*epoch;
    auto go = [&](auto fwd, auto mid, auto bwd, int nr) {
        hipLaunchKernelGGL(fwd, dim3(grid), dim3(64 * nr), 0, st, ys, ny, YF, YB, b, x, c, ran,
                           nchain, prog, ef);
        hipLaunchKernelGGL(mid, dim3(nstrips), dim3(64 * nr), 0, st, ys, ny, YF, YB, b, x, c);
        hipLaunchKernelGGL(bwd, dim3(grid), dim3(64 * nr), 0, st, ys, ny, YF, YB, x, c, nchain,
                           prog, eb);
    };
    if (max_nx <= 32)
        go(ysolve_fwd_kernel<4>, ysolve_mid_kernel<4>, ysolve_bwd_kernel<4>, 4);
    else if (max_nx <= 48)
        go(ysolve_fwd_kernel<6>, ysolve_mid_kernel<6>, ysolve_bwd_kernel<6>, 6);
    else if (max_nx <= 64)
        go(ysolve_fwd_kernel<8>, ysolve_mid_kernel<8>, ysolve_bwd_kernel<8>, 8);
    else
        return hipErrorInvalidValue;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, st);
    return e;
}
