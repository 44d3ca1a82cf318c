// The free interface operator L_h (Section 4.2, Proposition 3.1) applied in
// the eigenbasis of the y-direction.  With W = 0 the strip operator is the
// Kronecker sum K = A_x (x) M_y - c M_x (x) S_y (Section 2.2: Q1 mass and
// stiffness on the rectangular mesh; the Robin terms act on the strip's two
// x-edges only), and the 1-D pair (S_y, M_y) of a uniform mesh with free
// ends has the discrete cosines as generalised eigenvectors:
//     phi_mu(j) = alpha_mu cos(mu pi j / (ny - 1)),  S_y phi = lambda M_y phi,
//     lambda_mu = 6 (1 - cos th) / (hy^2 (2 + cos th)),  th = mu pi / (ny - 1),
// normalised to Phi^T M_y Phi = I, so Phi^{-1} = Phi^T M_y.  Every block of
// L_h is then Phi diag(.) Phi^{-1}: for strip class (nx, pl, pr) and mode mu,
// T_mu = A_x - c lambda_mu M_x (nx x nx, tridiagonal), and with t the corner
// entries of T_mu^{-1}
//     X^1 = 2ipc t_00 - 1,   X^2 = 2ipc t_{0,nx-1},
//     X^3 = 2ipc t_{nx-1,0}, X^4 = 2ipc t_{nx-1,nx-1} - 1   (per mode).
// A product L_h x is two dense real transforms of all 2(N-1) traces (one
// n x n matrix shared by all strips, on the FP64 matrix cores) around a
// per-mode 2 x 2 combination, instead of streaming ncls x 4 dense complex
// blocks.
#include "osm_internal.h"

namespace {

__device__ __forceinline__ v4d lhm_mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Input trace of output trace t (the pattern of eq. Lmpi): output 2i is the
// new r_i = X^1 l_{i+1} + X^2 r_{i+1} of strip i + 1, output 2i + 1 the new
// l_{i+1} = X^3 l_i + X^4 r_i of strip i; l_j is trace 2j - 1, r_j trace 2j
// (l_0 and r_{N-1} do not exist).
struct LhmSrc {
    int strip, bl, br, sl, sr;
};
__device__ __forceinline__ LhmSrc lhm_src(int t, int nsub) {
    LhmSrc s;
    const int i = t >> 1;
    if ((t & 1) == 0) {
        s.strip = i + 1; s.bl = 0; s.br = 1;
        s.sl = 2 * i + 1;
        s.sr = i + 1 <= nsub - 2 ? 2 * (i + 1) : -1;
    } else {
        s.strip = i; s.bl = 2; s.br = 3;
        s.sl = i >= 1 ? 2 * (i - 1) + 1 : -1;
        s.sr = 2 * i;
    }
    return s;
}

constexpr int TM_T = 16;   // traces per workgroup (32 real rows)
constexpr int TM_N = 64;   // output columns per workgroup
constexpr int TM_K = 64;   // k per staged block
constexpr int TM_QA = TM_T * TM_K / 256;   // complex inputs each thread stages per block
constexpr int TM_QB = TM_K * TM_N / 256;   // matrix entries each thread stages per block

// One staged block in registers.  Loads are unconditional, from indices
// clamped into the arrays (a load under a branch would make the compiler
// wait for every load in flight); store() zeroes what lies outside.
struct TmStage {
    double2 a[TM_QA];
    double b[TM_QB];
};

// out[t][r] = base[t][r] + sign sum_k Pm[r][k] a[t][k] for t < ntr, r < n
// (Pm real, row-major n x n; a, base, out complex, trace-major ntr x n).
// Real GEMM on the matrix cores: rows are (component, trace), wave w & 1
// takes the real or the imaginary parts, wave w >> 1 a pair of 16-column
// tiles; the blocks of k are staged through LDS, the next two in flight in
// registers while the current one is multiplied.
__global__ __launch_bounds__(256) void lhm_transform_kernel(int n, int ntr, const double *Pm,
                                                            const double2 *a,
                                                            const double2 *base, double sign,
                                                            double2 *out, const GmresCtl *ctl) {
    if (ctl && ctl->done) return;
    const int t0 = blockIdx.y * TM_T, r0 = blockIdx.x * TM_N;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int comp = wave & 1, nt0 = (wave >> 1) * 2;
    __shared__ double As[2][TM_T][TM_K + 1];    // [component][trace][k]
    __shared__ double Bs[TM_K][TM_N + 1];       // [k][column] = Pm[r0 + column][k0 + k]
    const int nkb = (n + TM_K - 1) / TM_K;
    auto load = [&](TmStage &st, int kb) {
        const int k0 = min(kb, nkb - 1) * TM_K;
#pragma unroll
        for (int q = 0; q < TM_QA; ++q) {
            const int e = tid + 256 * q, tt = e / TM_K, kk = e % TM_K;
            st.a[q] = a[(long)min(t0 + tt, ntr - 1) * n + min(k0 + kk, n - 1)];
        }
#pragma unroll
        for (int q = 0; q < TM_QB; ++q) {
            const int e = tid + 256 * q, rr = e / TM_K, kk = e % TM_K;
            st.b[q] = Pm[(long)min(r0 + rr, n - 1) * n + min(k0 + kk, n - 1)];
        }
    };
    auto store = [&](const TmStage &st, int kb) {
        const int k0 = kb * TM_K;
#pragma unroll
        for (int q = 0; q < TM_QA; ++q) {
            const int e = tid + 256 * q, tt = e / TM_K, kk = e % TM_K;
            const bool ok = t0 + tt < ntr && k0 + kk < n;
            As[0][tt][kk] = ok ? st.a[q].x : 0.0;
            As[1][tt][kk] = ok ? st.a[q].y : 0.0;
        }
#pragma unroll
        for (int q = 0; q < TM_QB; ++q) {
            const int e = tid + 256 * q, rr = e / TM_K, kk = e % TM_K;
            Bs[kk][rr] = (r0 + rr < n && k0 + kk < n) ? st.b[q] : 0.0;
        }
    };
    v4d acc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
    auto compute = [&]() {
#pragma unroll
        for (int ks = 0; ks < TM_K; ks += 4) {
            const double av = As[comp][lane & 15][ks + (lane >> 4)];
#pragma unroll
            for (int q = 0; q < 2; ++q)
                acc[q] = lhm_mfma(av, Bs[ks + (lane >> 4)][(nt0 + q) * 16 + (lane & 15)], acc[q]);
        }
    };
    TmStage s0, s1, s2;
    load(s0, 0);
    load(s1, 1);
    for (int kb = 0; kb < nkb; kb += 3) {
        store(s0, kb);
        __syncthreads();
        load(s2, kb + 2);
        compute();
        __syncthreads();
        if (kb + 1 >= nkb) break;
        store(s1, kb + 1);
        __syncthreads();
        load(s0, kb + 3);
        compute();
        __syncthreads();
        if (kb + 2 >= nkb) break;
        store(s2, kb + 2);
        __syncthreads();
        load(s1, kb + 4);
        compute();
        __syncthreads();
    }
    // lane holds rows (lane >> 4) + 4 v of each 16 x 16 tile, column lane & 15
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int t = t0 + (lane >> 4) + 4 * v, r = r0 + (nt0 + q) * 16 + (lane & 15);
            if (t < ntr && r < n) {
                double o = sign * acc[q][v];
                const long idx = (long)t * n + r;
                if (base) o += comp ? base[idx].y : base[idx].x;
                double *dst = reinterpret_cast<double *>(out + idx) + comp;
                *dst = o;
            }
        }
}

// yh[t][mu] = X^{bl}(mu) xh[sl][mu] + X^{br}(mu) xh[sr][mu]: the per-mode
// combination of output trace t's strip (its class's modal diagonals dm).
__global__ __launch_bounds__(256) void lhm_combine_kernel(int n, int nsub, const double2 *xh,
                                                          double2 *yh, const StripMeta *strips,
                                                          const double2 *dm,
                                                          const GmresCtl *ctl) {
    if (ctl && ctl->done) return;
    const int t = blockIdx.y;
    const int mu = blockIdx.x * blockDim.x + threadIdx.x;
    if (mu >= n) return;
    const LhmSrc s = lhm_src(t, nsub);
    const double2 *d = dm + (long)strips[s.strip].cls * 4 * n;
    double2 v = cd(0.0, 0.0);
    if (s.sl >= 0) v = cadd(v, cmul(d[(long)s.bl * n + mu], xh[(long)s.sl * n + mu]));
    if (s.sr >= 0) v = cadd(v, cmul(d[(long)s.br * n + mu], xh[(long)s.sr * n + mu]));
    yh[(long)t * n + mu] = v;
}

// ---------------------------------------------------------------- by FFT
// When n - 1 = N is a power of two the transforms are discrete cosine
// transforms of the first kind.  With z the even extension of a trace v to
// L = 2N points (z_j = v_j for j <= N, z_{L-j} = v_j), the DFT
// F(z)_mu = sum_j z_j exp(-2 pi i j mu / L) is even in mu and its first N + 1
// entries are sum_j c_j v_j cos(pi j mu / N) with c_j = 1 at the ends and 2
// inside.  The normalisation of Phi and the mass matrix cancel in the product
// Phi diag(d) Phi^{-1} = Phi diag(d) diag(mth) Phi^T D (M_y phi_mu =
// mth_mu D phi_mu, D = diag(1/2, 1, ..., 1, 1/2)): with alpha_mu^2 mth_mu
// times the end weights equal to 2/L, one block application is
//     X v = F(ext(d . F(ext v))) / L   on the entries 0..N,
// so L_h x needs one FFT of every trace and one of every output, with no
// matrix at all.  The FFT is Stockham's self-sorting radix-4 form (a radix-2
// pass first when log2 L is odd), in place in LDS: each pass reads its
// butterflies' inputs into registers, synchronises, then writes them to the
// sorted positions.
constexpr int FT_THREADS = 512;

// exp(-2 pi i m / L) for m < L from the quarter table tq[r], r < L/4
// (exp(-2 pi i q / 4) = (-i)^q for the quarter q of m).
__device__ __forceinline__ double2 ft_tw(const double2 *tq, int m, int lg) {
    const int q = m >> (lg - 2), r = m & ((1 << (lg - 2)) - 1);
    const double2 t = tq[r];
    if (q == 0) return t;
    if (q == 1) return cd(t.y, -t.x);
    if (q == 2) return cd(-t.x, -t.y);
    return cd(-t.y, t.x);
}

__device__ __forceinline__ void ft_table(double2 *tq, int lg) {
    const int q4 = 1 << (lg - 2);
    for (int r = threadIdx.x; r < q4; r += FT_THREADS) {
        double sn, cs;
        sincospi(ldexp((double)r, 1 - lg), &sn, &cs);     // angle 2 pi r / L
        tq[r] = cd(cs, -sn);
    }
}

// In-place DFT of buf[0..L), L = 2^lg, 3 <= lg <= 12.  Every pass has at
// most L/4 radix-4 (or, first, L/2 <= 1024 radix-2) butterflies: two per
// thread at most.
__device__ __forceinline__ void ft_fft(double2 *buf, const double2 *tq, int lg) {
    const int L = 1 << lg, tid = threadIdx.x;
    int ns = 1, lns = 0;
    for (int done = 0; done < lg;) {
        const bool r4 = ((lg - done) & 1) == 0;
        const int lr = r4 ? 2 : 1, B = L >> lr;
        double2 v[2][4];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int j = tid + q * FT_THREADS;
            if (j < B) {
                const int k = j & (ns - 1), step = lg - lns - lr;   // L / (ns R) = 2^step
                v[q][0] = buf[j];
                v[q][1] = cmul(buf[j + B], ft_tw(tq, k << step, lg));
                if (r4) {
                    v[q][2] = cmul(buf[j + 2 * B], ft_tw(tq, (2 * k) << step, lg));
                    v[q][3] = cmul(buf[j + 3 * B], ft_tw(tq, (3 * k) << step, lg));
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int j = tid + q * FT_THREADS;
            if (j < B) {
                const int k = j & (ns - 1), o = ((j - k) << lr) + k;
                if (r4) {
                    const double2 a0 = cadd(v[q][0], v[q][2]), a1 = csub(v[q][0], v[q][2]);
                    const double2 a2 = cadd(v[q][1], v[q][3]), d = csub(v[q][1], v[q][3]);
                    const double2 a3 = cd(d.y, -d.x);          // (v1 - v3) (-i)
                    buf[o] = cadd(a0, a2);
                    buf[o + ns] = cadd(a1, a3);
                    buf[o + 2 * ns] = csub(a0, a2);
                    buf[o + 3 * ns] = csub(a1, a3);
                } else {
                    buf[o] = cadd(v[q][0], v[q][1]);
                    buf[o + ns] = csub(v[q][0], v[q][1]);
                }
            }
        }
        __syncthreads();
        ns <<= lr;
        lns += lr;
        done += lr;
    }
}

// xh[t][mu] = F(ext x_t)_mu, mu <= N, for trace t = blockIdx.x.
__global__ __launch_bounds__(FT_THREADS) void lhf_forward_kernel(int n, int lg,
                                                                 const double2 *x, double2 *xh,
                                                                 const GmresCtl *ctl) {
    if (ctl && ctl->done) return;
    extern __shared__ double2 flds[];
    const int L = 1 << lg, N = n - 1, t = blockIdx.x;
    double2 *buf = flds, *tq = flds + L;
    ft_table(tq, lg);
    const double2 *xt = x + (long)t * n;
    for (int j = threadIdx.x; j <= N; j += FT_THREADS) {
        const double2 v = xt[j];
        buf[j] = v;
        if (j > 0 && j < N) buf[L - j] = v;
    }
    __syncthreads();
    ft_fft(buf, tq, lg);
    double2 *o = xh + (long)t * n;
    for (int mu = threadIdx.x; mu <= N; mu += FT_THREADS) o[mu] = buf[mu];
}

// Output trace t = blockIdx.x: its strip's per-mode combination of the
// transformed inputs, transformed back; out = base + sign y (base may be
// null; it may alias out).
__global__ __launch_bounds__(FT_THREADS) void lhf_inverse_kernel(
    int n, int lg, int nsub, const double2 *xh, const StripMeta *strips, const double2 *dm,
    const double2 *base, double sign, double2 *out, const GmresCtl *ctl) {
    if (ctl && ctl->done) return;
    extern __shared__ double2 flds[];
    const int L = 1 << lg, N = n - 1, t = blockIdx.x;
    double2 *buf = flds, *tq = flds + L;
    ft_table(tq, lg);
    const LhmSrc s = lhm_src(t, nsub);
    const double2 *d = dm + (long)strips[s.strip].cls * 4 * n;
    const double inv = ldexp(1.0, -lg);
    for (int mu = threadIdx.x; mu <= N; mu += FT_THREADS) {
        double2 v = cd(0.0, 0.0);
        if (s.sl >= 0) v = cadd(v, cmul(d[(long)s.bl * n + mu], xh[(long)s.sl * n + mu]));
        if (s.sr >= 0) v = cadd(v, cmul(d[(long)s.br * n + mu], xh[(long)s.sr * n + mu]));
        v = cd(v.x * inv, v.y * inv);
        buf[mu] = v;
        if (mu > 0 && mu < N) buf[L - mu] = v;
    }
    __syncthreads();
    ft_fft(buf, tq, lg);
    for (int j = threadIdx.x; j <= N; j += FT_THREADS) {
        const long idx = (long)t * n + j;
        const double2 y = buf[j];
        double2 o = cd(sign * y.x, sign * y.y);
        if (base) o = cadd(base[idx], o);
        out[idx] = o;
    }
}

// Dense block X^b of strip class cls: out[r][c] = sum_mu Phi[r][mu] d(mu)
// Phi^{-1}[mu][c] (for inspection; O(n^3)).
__global__ void lhm_dense_kernel(int n, const double *phi, const double *phinv,
                                 const double2 *d, double2 *out) {
    const int r = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double sr = 0.0, si = 0.0;
    for (int mu = 0; mu < n; ++mu) {
        const double w = phi[(long)r * n + mu] * phinv[(long)mu * n + c];
        sr += w * d[mu].x;
        si += w * d[mu].y;
    }
    out[(long)r * n + c] = cd(sr, si);
}

}  // namespace

hipError_t launch_lh_modal(hipStream_t st, const Phys &P, const StripMeta *strips,
                           const LhModal &md, const double2 *x, double2 *y, int mode_p,
                           const GmresCtl *ctl) {
    const int n = P.ny, ntr = 2 * (P.nsub - 1);
    if (md.lg > 0) {
        const size_t lds = lh_fft_lds(md.lg);
        hipLaunchKernelGGL(lhf_forward_kernel, dim3((unsigned)ntr), dim3(FT_THREADS), lds, st,
                           n, md.lg, x, md.xh, ctl);
        hipLaunchKernelGGL(lhf_inverse_kernel, dim3((unsigned)ntr), dim3(FT_THREADS), lds, st,
                           n, md.lg, P.nsub, (const double2 *)md.xh, strips, md.dm,
                           mode_p ? x : (const double2 *)nullptr, mode_p ? -1.0 : 1.0, y, ctl);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((n + TM_N - 1) / TM_N), (unsigned)((ntr + TM_T - 1) / TM_T));
    double2 *yh = md.xh + (long)ntr * n;
    // x^ = Phi^{-1} x for every trace
    hipLaunchKernelGGL(lhm_transform_kernel, grid, dim3(256), 0, st, n, ntr, md.phinv, x,
                       (const double2 *)nullptr, 1.0, md.xh, ctl);
    // the per-mode 2 x 2 combination of every strip's inputs
    hipLaunchKernelGGL(lhm_combine_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)ntr),
                       dim3(256), 0, st, n, P.nsub, (const double2 *)md.xh, yh, strips, md.dm,
                       ctl);
    // y = Phi y^, or x - that
    hipLaunchKernelGGL(lhm_transform_kernel, grid, dim3(256), 0, st, n, ntr, md.phi,
                       (const double2 *)yh, mode_p ? x : (const double2 *)nullptr,
                       mode_p ? -1.0 : 1.0, y, ctl);
    return hipGetLastError();
}

hipError_t launch_lh_modal_dense(hipStream_t st, int n, const LhModal &md, int cls, int blk,
                                 double2 *out) {
    hipLaunchKernelGGL(lhm_dense_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)n),
                       dim3(256), 0, st, n, md.phi, md.phinv, md.dm + ((long)cls * 4 + blk) * n,
                       out);
    return hipGetLastError();
}

size_t lh_fft_lds(int lg) { return ((size_t)5 << (lg - 2)) * sizeof(double2); }

int lh_fft_log2(int n) {
    const int N = n - 1;
    if (N < 4 || (N & (N - 1)) != 0) return 0;
    int lg = 1;
    while ((1 << (lg - 1)) < N) ++lg;          // L = 2N = 2^lg
    return lg <= 12 ? lg : 0;
}
