// Block-Thomas factorisation of the strip operators with dense ny x ny
// Schur complements (the strip system of eq. NproblemRobinNL ordered by
// x node-lines is block tridiagonal with tridiagonal blocks; K_j is complex
// symmetric, so the sub-diagonal block L_i equals U_{i-1}^T):
//     S_0 = D_0,   S_i = D_i - U_{i-1}^T S_{i-1}^{-1} U_{i-1}
// from above, and in the twisted form used by the strip solve also
//     T_{nx-1} = D_{nx-1},   T_i = D_i - U_i T_{i+1}^{-1} U_i^T
// from below, meeting at a middle line that eliminates both neighbours.
// Each S_i is inverted in place by a blocked symmetric sweep (Gauss-Jordan
// in the form that keeps the matrix symmetric) without pivoting: -i K_j has
// a positive definite Hermitian part (2/dt M + c p M^Gamma), so elimination
// without pivoting is well defined for every Schur complement, and S_i, its
// inverse and every intermediate of the sweep are complex symmetric.  The
// rank-128 updates run on the matrix cores (v_mfma_f64_16x16x4f64 /
// v_mfma_f32_16x16x4f32 on split real/imaginary tiles, complex products as
// three real products).
#include "osm_internal.h"

#include <algorithm>

#define SW 64    // tile edge of the sweep's updates and of the Schur complement
#define SB 128   // pivot block edge of the sweep (two tiles)

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
// lines' Schur complements (read through their upper triangles).  The
// complement is symmetric and the sweep reads only its upper 64 x 64 tiles
// (I <= J), so only those are formed.
// A tile is formed by SCHUR_QP workgroups, each on a band of
// 4 * SCHUR_RW rows; thread t owns column t % 64 and SCHUR_RW consecutive
// rows, sliding the three-row window of F U over them (short bands give
// many more waves to hide the loads' latency).
constexpr int SCHUR_RW = 4, SCHUR_QP = SW / (4 * SCHUR_RW);
template <typename T>
__global__ __launch_bounds__(256) void schur_kernel(int n, typename cplx_of<T>::type *F,
                                                    const int *lines, const int *kind,
                                                    const double2 *Dc, const double2 *Uc) {
    typedef typename cplx_of<T>::type T2;
    const int TT = (n + SW - 1) / SW, nt = TT * (TT + 1) / 2;
    const int z = blockIdx.x / (nt * SCHUR_QP), rest = blockIdx.x - z * nt * SCHUR_QP;
    const int qq = rest % SCHUR_QP;
    int I = 0, rem = rest / SCHUR_QP;
    while (rem >= TT - I) { rem -= TT - I; ++I; }
    const int J = I + rem;
    const int c = J * SW + (threadIdx.x & 63);
    const int rb = I * SW + qq * 4 * SCHUR_RW + (threadIdx.x >> 6) * SCHUR_RW;
    if (c >= n || rb >= n) return;
    const int re = min(rb + SCHUR_RW, n);
    const long L = lines[z];
    const int kd = kind[z];
    const long nn = (long)n * n;
    double2 acc[SCHUR_RW];
#pragma unroll
    for (int q = 0; q < SCHUR_RW; ++q) {
        const int r = rb + q;
        acc[q] = (r < n && abs(r - c) <= 1) ? Dc[(L * n + r) * 3 + (c - r + 1)] : cd(0.0, 0.0);
    }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        if (!(kd & (1 << side))) continue;
        // above: Lu = L-1, G = F_{L-1}, left factor U_{L-1}(a, r), right U_{L-1}(b, c)
        // below: Lu = L,   G = F_{L+1}, left factor U_L(r, a),   right U_L(c, b)
        const long Lu = side == 0 ? L - 1 : L;
        const T2 *G = F + (side == 0 ? L - 1 : L + 1) * nn;
        double2 ur[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int bb = c - 1 + d;
            ur[d] = cd(0.0, 0.0);
            if (bb >= 0 && bb < n)
                ur[d] = side == 0 ? Uc[(Lu * n + bb) * 3 + (c - bb + 1)]
                                  : Uc[(Lu * n + c) * 3 + (bb - c + 1)];
        }
        // t_a = sum_b G(a, b) U(b, c) for the window rows a = r-1, r, r+1
        auto trow = [&](int a) -> double2 {
            double2 t = cd(0.0, 0.0);
            if (a < 0 || a >= n) return t;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int bb = c - 1 + d;
                if (bb >= 0 && bb < n) {
                    // the neighbour's inverse may be stored as its upper
                    // triangle only: read G(a, bb) = G(min, max)
                    const int lo = min(a, bb), hi = max(a, bb);
                    const T2 g = G[(long)lo * n + hi];
                    t = cadd(t, cmul(cd(g.x, g.y), ur[d]));
                }
            }
            return t;
        };
        double2 tm = trow(rb - 1), t0 = trow(rb);
#pragma unroll
        for (int q = 0; q < SCHUR_RW; ++q) {
            const int r = rb + q;
            if (r < re) {
                const double2 tp = trow(r + 1);
                double2 sum = cd(0.0, 0.0);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int a = r - 1 + d;
                    if (a < 0 || a >= n) continue;
                    const double2 u = side == 0 ? Uc[(Lu * n + a) * 3 + (r - a + 1)]
                                                : Uc[(Lu * n + r) * 3 + (a - r + 1)];
                    sum = cadd(sum, cmul(u, d == 0 ? tm : (d == 1 ? t0 : tp)));
                }
                acc[q] = csub(acc[q], sum);
                tm = t0;
                t0 = tp;
            }
        }
    }
    T2 *S = F + L * nn;
#pragma unroll
    for (int q = 0; q < SCHUR_RW; ++q) {
        const int r = rb + q;
        if (r < re) S[(long)r * n + c] = mk2<T2>(acc[q].x, acc[q].y);
    }
}

// ---------------------------------------------------------------- sweep
// One pivot block K (rows/columns [k0, k0+b), b <= 128) of the symmetric
// sweep maps M to
//     M'[K,K] = -P,   M'[K,j] = P M[K,j],   M'[i,K] = M[i,K] P,
//     M'[i,j] = M[i,j] - M[i,K] P M[K,j],          P = M[K,K]^{-1},
// which keeps M symmetric; after every block has been swept M = -S^{-1}.
// Symmetry lets each pass compute and store only the upper 64 x 64 tiles
// (I <= J, the diagonal tiles in full); the last pass negates and also
// writes each off-diagonal tile's transpose, leaving the full inverse.
//   sweep_pivot_kernel   P of every line (one workgroup per line)
//   sweep_panel_kernel   C = M[K,:] before the pass, and R = P C
//   sweep_update_kernel  every upper tile: M[I,J] - C[:,I]^T R[:,J]

template <typename T> struct sweep_lds { static constexpr int LS = 80; };   // 80 words = 16 mod 32
template <> struct sweep_lds<double> { static constexpr int LS = 72; };     // 144 words = 16 mod 32

// LDS operand chunks of one 64 x 64 x KC product: a[k][i] = A(i, k),
// b[k][j] = B(k, j), real and imaginary parts split.
template <typename T>
struct SweepTile {
    static constexpr int KC = 32, LS = sweep_lds<T>::LS;
    T ar[KC][LS], ai[KC][LS], br[KC][LS], bi[KC][LS];
};

// A B over one chunk with three real products per complex product
// (Gauss): X += Ar Br, Y += Ai Bi, Z += (Ar + Ai)(Br + Bi), so that
// Re = X - Y and Im = Z - X - Y.  4 waves, 32 x 32 outputs each as 2 x 2
// blocks of 16 x 16 accumulators.
template <typename V4> struct Acc3 { V4 x[2][2], y[2][2], z[2][2]; };

template <typename T, typename V4>
__device__ __forceinline__ void sweep_mma(const SweepTile<T> &s, int lane, int wr, int wc,
                                          Acc3<V4> &a) {
    const int cl = lane & 15;
#pragma unroll
    for (int ks = 0; ks < SweepTile<T>::KC; ks += 4) {
        const int kr = ks + (lane >> 4);
        T a_r[2], a_i[2], a_s[2], b_r[2], b_i[2], b_s[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            a_r[q] = s.ar[kr][wr + q * 16 + cl];
            a_i[q] = s.ai[kr][wr + q * 16 + cl];
            b_r[q] = s.br[kr][wc + q * 16 + cl];
            b_i[q] = s.bi[kr][wc + q * 16 + cl];
            a_s[q] = a_r[q] + a_i[q];
            b_s[q] = b_r[q] + b_i[q];
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                a.x[bi][bj] = mfma16(a_r[bi], b_r[bj], a.x[bi][bj]);
                a.y[bi][bj] = mfma16(a_i[bi], b_i[bj], a.y[bi][bj]);
                a.z[bi][bj] = mfma16(a_s[bi], b_s[bj], a.z[bi][bj]);
            }
    }
}

// Accumulators holding base (re, im): X = re, Y = 0, Z = re + im.
template <typename T, typename V4>
__device__ __forceinline__ void acc3_set(Acc3<V4> &a, int bi, int bj, int v, T re, T im) {
    a.x[bi][bj][v] = re;
    a.y[bi][bj][v] = 0;
    a.z[bi][bj][v] = re + im;
}
template <typename T, typename V4>
__device__ __forceinline__ T acc3_re(const Acc3<V4> &a, int bi, int bj, int v) {
    return a.x[bi][bj][v] - a.y[bi][bj][v];
}
template <typename T, typename V4>
__device__ __forceinline__ T acc3_im(const Acc3<V4> &a, int bi, int bj, int v) {
    return a.z[bi][bj][v] - a.x[bi][bj][v] - a.y[bi][bj][v];
}

// P = M[K,K]^{-1} by in-place Gauss-Jordan on the 128 x 128 pivot block
// held in registers (thread t owns column t % 128 and rows t / 128 + 8 s);
// the pivot row and column of each step go through LDS (double-buffered,
// one barrier per pivot).  The block's lower off-diagonal 64-tile is not
// stored, so it is read from its mirror.  Identity-padded beyond b.  Stored
// k-major, Pbuf[z][k * 128 + i] = P(i, k), through LDS 32 rows at a time.
template <typename T>
__global__ __launch_bounds__(1024) void sweep_pivot_kernel(int n, int kb,
                                                           const typename cplx_of<T>::type *F,
                                                           const int *lines,
                                                           typename cplx_of<T>::type *Pbuf) {
    typedef typename cplx_of<T>::type T2;
    const int z = blockIdx.x, t = threadIdx.x;
    const int c = t & (SB - 1), g = t >> 7;
    const int k0 = kb * SB, b = min(SB, n - k0);
    const T2 *M = F + (long)lines[z] * n * (long)n;
    __shared__ T rowb[2][2][SB], colb[2][2][SB];
    __shared__ T tr[32][SB + 1], ti[32][SB + 1];
    T xr[16], xi[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int r = g + 8 * s;
        if (r < b && c < b) {
            const long idx = (r / SW > c / SW) ? (long)(k0 + c) * n + k0 + r
                                               : (long)(k0 + r) * n + k0 + c;
            const T2 v = M[idx];
            xr[s] = v.x; xi[s] = v.y;
        } else {
            xr[s] = (r == c) ? (T)1 : (T)0; xi[s] = 0;
        }
    }
    auto publish = [&](int p, int buf) {
        if (g == (p & 7)) {
#pragma unroll
            for (int s = 0; s < 16; ++s)
                if (s == (p >> 3)) { rowb[buf][0][c] = xr[s]; rowb[buf][1][c] = xi[s]; }
        }
        if (c == p) {
#pragma unroll
            for (int s = 0; s < 16; ++s) { colb[buf][0][g + 8 * s] = xr[s]; colb[buf][1][g + 8 * s] = xi[s]; }
        }
    };
    publish(0, 0);
    __syncthreads();
    for (int p = 0; p < b; ++p) {
        const int buf = p & 1;
        const T pr = rowb[buf][0][p], pim = rowb[buf][1][p];
        const T den = pr * pr + pim * pim;
        const T ivr = pr / den, ivi = -pim / den;
        const T rr = rowb[buf][0][c], ri = rowb[buf][1][c];
        const T qr = ivr * rr - ivi * ri, qi = ivr * ri + ivi * rr;     // a_pc / a_pp
        // branch-free: column p takes -a_rp / a_pp, row p takes a_pc / a_pp
        // (1 / a_pp on the diagonal), every other element a_rc - a_rp a_pc / a_pp
        const bool isc = c == p, rowp = g == (p & 7);
        const int sp = p >> 3;
        const T hr = isc ? ivr : qr, hi = isc ? ivi : qi;
        const T mr = isc ? ivr : qr, mi = isc ? ivi : qi;   // multiplier of a_rp
        const T kx = isc ? (T)0 : (T)1;                    // keep a_rc off column p
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const T cr = colb[buf][0][g + 8 * s], ci = colb[buf][1][g + 8 * s];   // a_rp
            T nr = kx * xr[s] - (cr * mr - ci * mi);
            T ni = kx * xi[s] - (cr * mi + ci * mr);
            const bool hit = rowp && s == sp;
            xr[s] = hit ? hr : nr;
            xi[s] = hit ? hi : ni;
        }
        if (p + 1 < b) publish(p + 1, buf ^ 1);
        __syncthreads();
    }
    T2 *P = Pbuf + (long)z * SB * SB;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            const int s = 4 * q + s2;               // rows g + 8 s lie in [32 q, 32 q + 32)
            tr[g + 8 * s - 32 * q][c] = xr[s];
            ti[g + 8 * s - 32 * q][c] = xi[s];
        }
        __syncthreads();
        for (int e = t; e < 32 * SB; e += 1024) {
            const int i = e & 31, k = e >> 5;
            P[(long)k * SB + 32 * q + i] = mk2<T2>(tr[i][k], ti[i][k]);
        }
        __syncthreads();
    }
}

// Panel of pivot block kb for column tile J and row half rh of line z: the
// raw pivot rows C[k][j] = M[k0 + k][j] (read from the stored upper tiles
// (J, .) when J lies left of the block; written by the rh = 0 workgroup)
// and R[rh * 64 + r][j] = (P C)(rh * 64 + r, j); on the block's own columns
// R = P.  Rbuf, Cbuf: 128 x n per line.
template <typename T>
__global__ __launch_bounds__(256) void sweep_panel_kernel(int n, int kb,
                                                          const typename cplx_of<T>::type *F,
                                                          const int *lines,
                                                          const typename cplx_of<T>::type *Pbuf,
                                                          typename cplx_of<T>::type *Rbuf,
                                                          typename cplx_of<T>::type *Cbuf) {
    typedef typename cplx_of<T>::type T2;
    typedef typename vec4_of<T>::type V4;
    constexpr int KC = SweepTile<T>::KC;
    const int J = blockIdx.x, rh = blockIdx.y, z = blockIdx.z, tid = threadIdx.x;
    const int k0 = kb * SB, b = min(SB, n - k0);
    const int kt0 = k0 / SW, nbt = (b + SW - 1) / SW;
    const int j0 = J * SW, w = min(SW, n - j0);
    const int r0 = rh * SW;
    if (r0 >= b) return;
    const int hr = min(SW, b - r0);
    const T2 *M = F + (long)lines[z] * n * (long)n;
    const T2 *P = Pbuf + (long)z * SB * SB;
    T2 *R = Rbuf + (long)z * SB * n;
    T2 *C = Cbuf + (long)z * SB * n;
    if (J >= kt0 && J < kt0 + nbt) {
        const int c0 = j0 - k0;
        for (int e = tid; e < SW * SW; e += 256) {
            const int r = e >> 6, cc = e & 63;
            if (r < hr && cc < w) R[(long)(r0 + r) * n + j0 + cc] = P[(long)(c0 + cc) * SB + r0 + r];
        }
        return;
    }
    __shared__ SweepTile<T> sh;
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    Acc3<V4> acc;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc3_set<T, V4>(acc, bi, bj, v, (T)0, (T)0);
    for (int kc = 0; kc < b; kc += KC) {
        for (int e = tid; e < KC * SW; e += 256) {
            const int kk = e >> 6, i = e & 63;
            const T2 v = P[(long)(kc + kk) * SB + r0 + i];   // rows kc+kk >= b meet zero C rows
            sh.ar[kk][i] = v.x; sh.ai[kk][i] = v.y;
        }
        if (J > kt0) {
            for (int e = tid; e < KC * SW; e += 256) {
                const int kk = e >> 6, j = e & 63;
                T2 v;
                if (kc + kk < b && j < w) v = M[(long)(k0 + kc + kk) * n + j0 + j];
                else { v.x = 0; v.y = 0; }
                sh.br[kk][j] = v.x; sh.bi[kk][j] = v.y;
            }
        } else {
            for (int e = tid; e < KC * SW; e += 256) {
                const int j = e / KC, kk = e % KC;
                T2 v;
                if (kc + kk < b && j < w) v = M[(long)(j0 + j) * n + k0 + kc + kk];
                else { v.x = 0; v.y = 0; }
                sh.br[kk][j] = v.x; sh.bi[kk][j] = v.y;
            }
        }
        __syncthreads();
        if (rh == 0) {
            for (int e = tid; e < KC * SW; e += 256) {
                const int kk = e >> 6, j = e & 63;
                if (kc + kk < b && j < w)
                    C[(long)(kc + kk) * n + j0 + j] = mk2<T2>(sh.br[kk][j], sh.bi[kk][j]);
            }
        }
        sweep_mma<T, V4>(sh, lane, wr, wc, acc);
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wr + bi * 16 + acc_row<T>(lane, v);
                const int j = wc + bj * 16 + (lane & 15);
                if (r < hr && j < w)
                    R[(long)(r0 + r) * n + j0 + j] = mk2<T2>(acc3_re<T, V4>(acc, bi, bj, v),
                                                             acc3_im<T, V4>(acc, bi, bj, v));
            }
}

// Upper tiles (I <= J) of every line after pivot block kb.  Lines are
// spread over the 8 XCDs by blockIdx % 8 (a line's tiles share its panels,
// so they stay in one XCD's L2) when the batch has 8 lines or more.  The
// next chunk of C and R is loaded into registers while the current one is
// multiplied, and the tile's old value is added at the end.  On the last
// pass (last != 0) the result is negated, and with mirror != 0 (only on the
// last pass) off-diagonal tiles are also written transposed.
template <typename T>
__global__ __launch_bounds__(256) void sweep_update_kernel(int n, int kb,
                                                           typename cplx_of<T>::type *F,
                                                           const int *lines, int bt,
                                                           const typename cplx_of<T>::type *Rbuf,
                                                           const typename cplx_of<T>::type *Cbuf,
                                                           int last, int mirror) {
    typedef typename cplx_of<T>::type T2;
    typedef typename vec4_of<T>::type V4;
    constexpr int KC = SweepTile<T>::KC;
    const int TT = (n + SW - 1) / SW, nt = TT * (TT + 1) / 2;
    int z, t;
    if (bt >= 8) {
        const int x = blockIdx.x & 7, sidx = blockIdx.x >> 3;
        const int li = sidx / nt;
        t = sidx - li * nt;
        z = li * 8 + x;
        if (z >= bt) return;
    } else {
        z = blockIdx.x / nt;
        t = blockIdx.x - z * nt;
    }
    int I = 0, rem = t;
    while (rem >= TT - I) { rem -= TT - I; ++I; }
    const int J = I + rem;
    const int i0 = I * SW, j0 = J * SW, h = min(SW, n - i0), w = min(SW, n - j0);
    const int k0 = kb * SB, b = min(SB, n - k0);
    const int kt0 = k0 / SW, nbt = (b + SW - 1) / SW;
    const bool inI = I >= kt0 && I < kt0 + nbt, inJ = J >= kt0 && J < kt0 + nbt;
    T2 *M = F + (long)lines[z] * n * (long)n;
    const T2 *R = Rbuf + (long)z * SB * n;
    const T2 *C = Cbuf + (long)z * SB * n;
    const T so = last ? (T)-1 : (T)1;
    const int tid = threadIdx.x;
    __shared__ SweepTile<T> sh;
    if (inI) {
        // pivot rows: R (and -P on the block's own tiles)
        const T f = inJ ? -so : so;
        const int rr = (I - kt0) * SW;
        for (int e = tid; e < SW * SW; e += 256) {
            const int r = e >> 6, cc = e & 63;
            if (r < h && cc < w) {
                T2 v = R[(long)(rr + r) * n + j0 + cc];
                v.x *= f; v.y *= f;
                M[(long)(i0 + r) * n + j0 + cc] = v;
                if (mirror && J != I) M[(long)(j0 + cc) * n + i0 + r] = v;
            }
        }
        return;
    }
    if (inJ) {
        // pivot columns: M'[i, j] = R[j - k0][i]
        const int rc = (J - kt0) * SW;
        for (int jc = 0; jc < w; jc += KC) {
            for (int e = tid; e < KC * SW; e += 256) {
                const int jj = e >> 6, i = e & 63;
                T2 v;
                if (jc + jj < w && i < h) v = R[(long)(rc + jc + jj) * n + i0 + i];
                else { v.x = 0; v.y = 0; }
                sh.ar[jj][i] = so * v.x; sh.ai[jj][i] = so * v.y;
            }
            __syncthreads();
            for (int e = tid; e < KC * SW; e += 256) {
                const int i = e / KC, jj = e % KC;
                if (jc + jj < w && i < h)
                    M[(long)(i0 + i) * n + j0 + jc + jj] = mk2<T2>(sh.ar[jj][i], sh.ai[jj][i]);
            }
            if (mirror) {
                for (int e = tid; e < KC * SW; e += 256) {
                    const int jj = e >> 6, i = e & 63;
                    if (jc + jj < w && i < h)
                        M[(long)(j0 + jc + jj) * n + i0 + i] = mk2<T2>(sh.ar[jj][i], sh.ai[jj][i]);
                }
            }
            __syncthreads();
        }
        return;
    }
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    constexpr int PER = KC * SW / 256;
    T2 ra[PER], rb[PER];
    auto load = [&](int kc) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q, kk = e >> 6, i = e & 63;
            const bool ok = kc + kk < b;
            const int o = (kc + kk) * n;                // < 128 n: 32-bit offsets
            if (ok && i < h) ra[q] = C[o + i0 + i];
            else { ra[q].x = 0; ra[q].y = 0; }
            if (ok && i < w) rb[q] = R[o + j0 + i];
            else { rb[q].x = 0; rb[q].y = 0; }
        }
    };
    load(0);
    T2 base[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wr + bi * 16 + acc_row<T>(lane, v);
                const int j = wc + bj * 16 + (lane & 15);
                if (r < h && j < w) base[bi][bj][v] = M[(i0 + r) * n + j0 + j];   // n^2 < 2^31
                else { base[bi][bj][v].x = 0; base[bi][bj][v].y = 0; }
            }
    Acc3<V4> acc;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc3_set<T, V4>(acc, bi, bj, v, (T)0, (T)0);
    for (int kc = 0; kc < b; kc += KC) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q, kk = e >> 6, i = e & 63;
            sh.ar[kk][i] = -ra[q].x; sh.ai[kk][i] = -ra[q].y;
            sh.br[kk][i] = rb[q].x; sh.bi[kk][i] = rb[q].y;
        }
        __syncthreads();
        if (kc + KC < b) load(kc + KC);
        sweep_mma<T, V4>(sh, lane, wr, wc, acc);
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wr + bi * 16 + acc_row<T>(lane, v);
                const int j = wc + bj * 16 + (lane & 15);
                if (r < h && j < w) {
                    const T2 o = mk2<T2>(so * (base[bi][bj][v].x + acc3_re<T, V4>(acc, bi, bj, v)),
                                         so * (base[bi][bj][v].y + acc3_im<T, V4>(acc, bi, bj, v)));
                    M[(i0 + r) * n + j0 + j] = o;
                    if (mirror && I != J) M[(j0 + j) * n + i0 + r] = o;
                }
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
    const int TT = (n + SW - 1) / SW;
    const long blocks = (long)batch * (TT * (TT + 1) / 2) * SCHUR_QP;
    if (blocks > 0x7fffffffL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(schur_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, n, F, lines,
                       kind, Dc, Uc);
    return hipGetLastError();
}

int sweep_passes(int n) { return (n + SB - 1) / SB; }

// Algorithmic flops of one line's update in pass kb: 8 real flops per complex
// multiply-add over the upper tiles outside the pivot block's rows and
// columns (the kernel forms three real products per complex one).
double sweep_pass_flops(int n, int kb) {
    const int TT = (n + SW - 1) / SW, k0 = kb * SB, b = std::min(SB, n - k0);
    const int kt0 = k0 / SW, nbt = (b + SW - 1) / SW;
    double macs = 0.0;
    for (int I = 0; I < TT; ++I) {
        if (I >= kt0 && I < kt0 + nbt) continue;
        const double h = std::min(SW, n - I * SW);
        for (int J = I; J < TT; ++J) {
            if (J >= kt0 && J < kt0 + nbt) continue;
            macs += h * std::min(SW, n - J * SW) * (double)b;
        }
    }
    return 8.0 * macs;
}

// One pass of the sweep over lines[0..batch): pivot inverses, panels, then
// the update (bracketed by ev0/ev1 when given).  full != 0: the last pass
// also writes the lower triangles (full storage); else the inverses keep
// only their upper 64 x 64 tiles.
template <typename T>
hipError_t launch_sweep_pass(hipStream_t st, int n, int kb, typename cplx_of<T>::type *F,
                             const int *lines, int batch, typename cplx_of<T>::type *Pbuf,
                             typename cplx_of<T>::type *Rbuf, typename cplx_of<T>::type *Cbuf,
                             int full, hipEvent_t ev0, hipEvent_t ev1) {
    typedef typename cplx_of<T>::type T2;
    const int TT = (n + SW - 1) / SW, nt = TT * (TT + 1) / 2, passes = sweep_passes(n);
    const long ublocks = batch >= 8 ? 8L * ((batch + 7) / 8) * nt : (long)batch * nt;
    if (ublocks > 0x7fffffffL || batch > 65535 || kb < 0 || kb >= passes)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(sweep_pivot_kernel<T>, dim3(batch), dim3(1024), 0, st, n, kb,
                       (const T2 *)F, lines, Pbuf);
    hipLaunchKernelGGL(sweep_panel_kernel<T>, dim3(TT, 2, batch), dim3(256), 0, st, n, kb,
                       (const T2 *)F, lines, (const T2 *)Pbuf, Rbuf, Cbuf);
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(sweep_update_kernel<T>, dim3((unsigned)ublocks), dim3(256), 0, st, n, kb,
                       F, lines, batch, (const T2 *)Rbuf, (const T2 *)Cbuf,
                       kb == passes - 1 ? 1 : 0, (kb == passes - 1 && full) ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
    return hipSuccess;
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
template hipError_t launch_sweep_pass<double>(hipStream_t, int, int, double2 *, const int *, int,
                                              double2 *, double2 *, double2 *, int, hipEvent_t,
                                              hipEvent_t);
template hipError_t launch_sweep_pass<float>(hipStream_t, int, int, float2 *, const int *, int,
                                             float2 *, float2 *, float2 *, int, hipEvent_t,
                                             hipEvent_t);
template hipError_t launch_zgemm<double>(hipStream_t, const GemmArgs<double> &, int);
template hipError_t launch_zgemm<float>(hipStream_t, const GemmArgs<float> &, int);
template hipError_t launch_convert<double>(hipStream_t, long, const double2 *, double2 *);
template hipError_t launch_convert<float>(hipStream_t, long, const double2 *, float2 *);
