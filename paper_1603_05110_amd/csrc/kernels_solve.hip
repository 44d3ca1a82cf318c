// Block-tridiagonal substitution with the stored inverses of the twisted
// factor, for every strip at once.  A strip with nx lines has its middle line
// m = (nx-1)/2: lines above it hold S_i^{-1} (eliminated from above), lines
// below hold T_i^{-1} (eliminated from below), line m holds the inverse of
// the Schur complement that eliminates both neighbours.  The solve runs
//   forward   y_i = S_i^{-1} (b_i - U_{i-1}^T y_{i-1})      i = 0 .. m-1
//             z_i = T_i^{-1} (b_i - U_i z_{i+1})            i = nx-1 .. m+1
//   middle    x_m = Z^{-1} (b_m - U_{m-1}^T y_{m-1} - U_m z_{m+1})
//   backward  x_i = y_i - S_i^{-1} U_i x_{i+1}               i = m-1 .. 0
//             x_i = z_i - T_i^{-1} U_{i-1}^T x_{i-1}         i = m+1 .. nx-1
// with one line from above and one from below per step: nx + 1 dependent
// steps (nx odd) instead of 2 nx - 1.  This is the local solve that the fixed
// point, the classical iteration and every outer preconditioned iteration
// repeat (Section 2.2, eq. NproblemRobinNL; Section 5: LU solves of the strip
// systems).  Each product is a dense ny x ny matrix-vector product streamed
// from HBM, so the kernel is bandwidth-bound.
//
// Launch: one persistent cooperative grid, `team` workgroups per strip; the
// workgroup with blockIdx b serves strip b % nstrips (so with a strip count
// that is a multiple of 8 a strip's team sits on one XCD) and owns a
// contiguous row range of every product.  Consecutive steps of a strip are
// ordered by a per-strip counter barrier: stores drained, one relaxed
// device-scope increment by the arriving workgroup, relaxed polling, rows
// exchanged with device-coherent loads.  The wait is bounded and sets an
// error flag, so no wave can spin forever.
#include "step_bodies.h"

namespace {

constexpr int SOLVE_THREADS = 256;
constexpr unsigned SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ void team_barrier(unsigned *ctr, unsigned target, int *err) {
    __builtin_amdgcn_s_waitcnt(0);   // this wave's stores are acknowledged
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // publish the workgroup's rows
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > SPIN_LIMIT ||
                __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

template <typename T> struct acc_t;
template <> struct acc_t<double> { typedef double type; };
template <> struct acc_t<float> { typedef float type; };

// Agent-scope (device-coherent) stores and loads of one complex value: the
// vectors exchanged between the workgroups of a team go through these, so
// the barrier needs no cache-wide writeback or invalidation.
__device__ __forceinline__ void st_agent(double2 *p, double2 v) {
    double *d = reinterpret_cast<double *>(p);
    __hip_atomic_store(d, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(d + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double2 ld_agent(const double2 *p) {
    const double *d = reinterpret_cast<const double *>(p);
    return cd(__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
              __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// ---------------------------------------------------------------- twisted schedule
enum { TOP_F = 0, BOT_F = 1, MID = 2, TOP_B = 3, BOT_B = 4 };

// Products of step s of a strip with nx lines: local line and kind of the
// product from above (lt) and from below (lb); -1 = none.
struct TwStep {
    int lt, kt, lb, kb;
};

__device__ __forceinline__ int tw_steps(int nx) { return 2 * (nx - 1 - (nx - 1) / 2) + 1; }

__device__ __forceinline__ TwStep tw_step(int nx, int s) {
    const int m = (nx - 1) / 2, nb = nx - 1 - m;
    TwStep t;
    if (s < nb) {
        t.lt = s < m ? s : -1; t.kt = TOP_F;
        t.lb = nx - 1 - s;     t.kb = BOT_F;
    } else if (s == nb) {
        t.lt = m;  t.kt = MID;
        t.lb = -1; t.kb = BOT_F;
    } else {
        int e = s - nb - 1;
        t.lt = m - 1 - e >= 0 ? m - 1 - e : -1; t.kt = TOP_B;
        t.lb = m + 1 + e;                        t.kb = BOT_B;
    }
    return t;
}

__device__ __forceinline__ bool tw_backward(int kind) { return kind == TOP_B || kind == BOT_B; }

// Element r of the vector a product multiplies, in FP64: b_i minus (forward,
// middle) or plus (backward) the coupling terms U_{i-1}^T x_{i-1} ("up") and
// U_i x_{i+1} ("down") with the neighbouring lines' rows; L is the packed
// line, i = L - (strip's first line).  xl(line, q) loads x[line * n + q].
template <class XL>
__device__ __forceinline__ double2 tw_vec(int kind, long L, int i, int nx, int n, int r,
                                          const double2 *b, const double2 *Uc, XL xl) {
    double2 acc = cd(0.0, 0.0);
    bool up = false, down = false;
    if (kind == TOP_F) { acc = b[L * n + r]; up = i > 0; }
    else if (kind == BOT_F) { acc = b[L * n + r]; down = i < nx - 1; }
    else if (kind == MID) { acc = b[L * n + r]; up = true; down = true; }
    else if (kind == TOP_B) down = true;
    else up = true;
    const double sg = tw_backward(kind) ? 1.0 : -1.0;
    if (up) {
        double2 cu[3], xv[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int q = r - 1 + d;
            bool ok = q >= 0 && q < n;
            cu[d] = ok ? Uc[((L - 1) * n + q) * 3 + (2 - d)] : cd(0.0, 0.0);   // U_{i-1}(q, r)
            xv[d] = ok ? xl(L - 1, q) : cd(0.0, 0.0);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) acc = cadd(acc, cscale(sg, cmul(cu[d], xv[d])));
    }
    if (down) {
        double2 cu[3], xv[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int q = r - 1 + d;
            bool ok = q >= 0 && q < n;
            cu[d] = ok ? Uc[(L * n + r) * 3 + d] : cd(0.0, 0.0);               // U_i(r, q)
            xv[d] = ok ? xl(L + 1, q) : cd(0.0, 0.0);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) acc = cadd(acc, cscale(sg, cmul(cu[d], xv[d])));
    }
    return acc;
}

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_f64(v); }
__device__ __forceinline__ float wave_sum(float v) { return wave_sum_f32(v); }

// out[r] = sum_c M[r][c] vec[c] for rows r in [r0, r1) of one workgroup.
// Wave w takes rows r0 + w, r0 + w + 4, ...; RU of its rows at a time, and
// UN column chunks of 64 per pass, all loads issued before the FMAs.
// mode 0: x[r] = out; mode 1: x[r] -= out.
template <typename T, int RU, int UN>
__device__ __forceinline__ void wg_gemv(const typename cplx_of<T>::type *__restrict__ M, int n,
                                        int r0, int r1, const typename cplx_of<T>::type *vec,
                                        double2 *__restrict__ x, int mode, double inv) {
    typedef typename cplx_of<T>::type T2;
    typedef typename acc_t<T>::type A;
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int rb = r0 + wave; rb < r1; rb += 4 * RU) {
        A ar[RU], ai[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) { ar[u] = 0; ai[u] = 0; }
        for (int c0 = 0; c0 < n; c0 += 64 * UN) {
            T2 m[RU][UN];
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int k = 0; k < UN; ++k) {
                    int r = rb + 4 * u, c = c0 + lane + 64 * k;
                    if (r < r1 && c < n) m[u][k] = M[(long)r * n + c];
                    else { m[u][k].x = 0; m[u][k].y = 0; }
                }
#pragma unroll
            for (int k = 0; k < UN; ++k) {
                int c = c0 + lane + 64 * k;
                T2 v;
                if (c < n) v = vec[c];
                else { v.x = 0; v.y = 0; }
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    ar[u] += m[u][k].x * v.x - m[u][k].y * v.y;
                    ai[u] += m[u][k].x * v.y + m[u][k].y * v.x;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            A sr = wave_sum(ar[u]);
            A si = wave_sum(ai[u]);
            int r = rb + 4 * u;
            if (lane == 0 && r < r1) {
                if (mode == 0) x[r] = cd((double)sr * inv, (double)si * inv);
                else {
                    double2 o = x[r];
                    x[r] = cd(o.x - (double)sr * inv, o.y - (double)si * inv);
                }
            }
        }
    }
}

template <typename T> struct tile_shape;
template <> struct tile_shape<float> { static constexpr int RU = 2, UN = 8; };
template <> struct tile_shape<double> { static constexpr int RU = 2, UN = 4; };

// Power of two s with 1 <= s * (largest |b| of the strip) < 2 (1 when the
// right-hand side is zero or not finite); every lane reads the same nx line
// maxima, so no exchange is needed.
__device__ __forceinline__ double strip_scale(const double *lm, int nx) {
    if (!lm) return 1.0;
    double mx = 0.0;
    for (int i = 0; i < nx; ++i) mx = fmax(mx, lm[i]);
    return (mx > 0.0 && isfinite(mx)) ? ldexp(1.0, -ilogb(mx)) : 1.0;
}

__device__ __forceinline__ bool solve_skipped(const SolveArgs &a) {
    bool skip = a.ctl && (a.ctl->q_conv || a.ctl->k_done || a.ctl->bad);
    if (!skip && a.ran && blockIdx.x == 0 && threadIdx.x == 0) *a.ran = 1;
    return skip;
}

template <typename T>
__global__ __launch_bounds__(SOLVE_THREADS) void strip_solve_kernel(SolveArgs a) {
    typedef typename cplx_of<T>::type T2;
    constexpr int RU = tile_shape<T>::RU, UN = tile_shape<T>::UN;
    if (solve_skipped(a)) return;
    extern __shared__ unsigned char smem_raw[];
    T2 *vecs = reinterpret_cast<T2 *>(smem_raw);   // 2 n: product from above, from below
    int nst = a.nstrips, team = a.team;
    int j = blockIdx.x % nst, w = blockIdx.x / nst;
    StripMeta s = a.strips[j];
    int n = a.n;
    int rpw = (n + team - 1) / team;
    int r0 = min(n, w * rpw), r1 = min(n, r0 + rpw);
    const T2 *F = reinterpret_cast<const T2 *>(a.F);
    unsigned *ctr = a.counters + j;
    unsigned epoch = 0;
    const long nn = (long)n * n;
    const double sc = strip_scale(a.lmax ? a.lmax + s.off : nullptr, s.nx), inv = 1.0 / sc;
    auto xl = [&](long line, int q) -> double2 { return ld_agent(a.x + line * n + q); };
    const int S = tw_steps(s.nx);
    for (int st = 0; st < S; ++st) {
        const TwStep t = tw_step(s.nx, st);
        
        for (int p = 0; p < 2; ++p) {
            if ((p == 0 ? t.lt : t.lb) < 0) continue;
            long L = s.off + (p == 0 ? t.lt : t.lb);
            for (int r = threadIdx.x; r < n; r += SOLVE_THREADS) {
                double2 v = tw_vec((p == 0 ? t.kt : t.kb), L, (p == 0 ? t.lt : t.lb), s.nx, n, r, a.b, a.Uc, xl);
                T2 tv; tv.x = (T)(v.x * sc); tv.y = (T)(v.y * sc);
                vecs[p * n + r] = tv;
            }
        }
        __syncthreads();
        for (int p = 0; p < 2; ++p) {
            if ((p == 0 ? t.lt : t.lb) < 0) continue;
            long L = s.off + (p == 0 ? t.lt : t.lb);
            wg_gemv<T, RU, UN>(F + L * nn, n, r0, r1, vecs + p * n, a.x + L * n,
                               tw_backward((p == 0 ? t.kt : t.kb)) ? 1 : 0, inv);
        }
        if (st == S - 1) break;
        team_barrier(ctr, (++epoch) * team, a.error);
        if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    }
}

// Prefetching variant for ny <= 64 NCH.  A step's rows of both products
// form one list (the rows [r0, r1) of the product from above, then of the
// product from below), dealt round-robin to the NW waves; each wave keeps its
// first PR rows, NCH column chunks of 64, in registers.  Right after the
// workgroup has published a step and arrived at the strip barrier, it loads
// its rows of the next step (the stored inverses do not depend on the
// vectors), so the HBM stream overlaps the barrier wait and the next vector
// phase.
template <typename T, int NW, int NCH, int PR>
__global__ __launch_bounds__(NW * 64) void strip_solve_pf_kernel(SolveArgs a) {
    typedef typename cplx_of<T>::type T2;
    typedef typename acc_t<T>::type A;
    if (solve_skipped(a)) return;
    extern __shared__ unsigned char smem_raw[];
    T2 *vecs = reinterpret_cast<T2 *>(smem_raw);   // 2 n: product from above, from below
    constexpr int NTHR = NW * 64;
    const int nst = a.nstrips, team = a.team;
    const int j = blockIdx.x % nst, w = blockIdx.x / nst;
    const StripMeta s = a.strips[j];
    const int n = a.n;
    const int rpw = (n + team - 1) / team;
    const int r0 = min(n, w * rpw), r1 = min(n, r0 + rpw), R = r1 - r0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const T2 *F = reinterpret_cast<const T2 *>(a.F);
    unsigned *ctr = a.counters + j;
    const long nn = (long)n * n;
    const int S = tw_steps(s.nx);
    // 2 n after vecs: forward results of this member's rows of the step's
    // backward lines, loaded while the team barrier is pending, so that a
    // backward row does not wait for a device-coherent load when it is
    // finished.  (The one-row tiles need the library built without IR-level
    // common-code sinking: it merged the last store of the two finish_row
    // call sites below, and the structurized loop then ran its wave sums
    // with lane 0 masked off.)
    double2 *ofwd = reinterpret_cast<double2 *>(vecs + 2 * n);
    TwStep t = tw_step(s.nx, 0);
    const double sc = strip_scale(a.lmax ? a.lmax + s.off : nullptr, s.nx), inv = 1.0 / sc;
    T2 m[PR][NCH];

    // entry rho of a step's row list -> product p (0 above, 1 below) and row
    // r, packed as p * 65536 + r; -1 past the end
    auto entry = [&](const TwStep &t, int rho) -> int {
        if (t.lt >= 0) {
            if (rho < R) return r0 + rho;
            rho -= R;
        }
        if (t.lb >= 0 && rho < R) return 65536 + r0 + rho;
        return -1;
    };
    auto line_of = [&](const TwStep &t, int p) -> long { return s.off + (p == 0 ? t.lt : t.lb); };
    auto prefetch = [&](const TwStep &t) {
#pragma unroll
        for (int u = 0; u < PR; ++u) {
            const int e = entry(t, wave + NW * u);
            const bool ok = e >= 0;
            const int p = e >> 16, r = e & 0xFFFF;
            const T2 *M = ok ? F + line_of(t, p) * nn + (long)r * n : F;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                int col = c * 64 + lane;
                if (ok && col < n) m[u][c] = M[col];
                else { m[u][c].x = 0; m[u][c].y = 0; }
            }
        }
    };
    auto finish_row = [&](long L, int r, bool bwd, A ar, A ai) {
        ar = wave_sum(ar);
        ai = wave_sum(ai);
        if (lane == 0) {
            double2 *xr = a.x + L * n + r;
            if (!bwd) st_agent(xr, cd((double)ar * inv, (double)ai * inv));
            else {
                const int p = (t.lt >= 0 && L == line_of(t, 0)) ? 0 : 1;
                const double2 o = ofwd[p * n + (r - r0)];
                st_agent(xr, cd(o.x - (double)ar * inv, o.y - (double)ai * inv));
            }
        }
    };
    auto xl = [&](long line, int q) -> double2 { return ld_agent(a.x + line * n + q); };
    auto prefetch_o = [&](const TwStep &tn) {
        for (int p = 0; p < 2; ++p) {
            if ((p == 0 ? tn.lt : tn.lb) < 0 || !tw_backward(p == 0 ? tn.kt : tn.kb)) continue;
            const long L = line_of(tn, p);
            for (int q = threadIdx.x; q < R; q += NTHR) ofwd[p * n + q] = ld_agent(a.x + L * n + r0 + q);
        }
    };

    prefetch(t);
    for (int st = 0; st < S; ++st) {
        
        // vector phase: both products' vectors, all loads of an entry issued together
        for (int p = 0; p < 2; ++p) {
            if ((p == 0 ? t.lt : t.lb) < 0) continue;
            const long L = s.off + (p == 0 ? t.lt : t.lb);
            for (int r = threadIdx.x; r < n; r += NTHR) {
                double2 v = tw_vec((p == 0 ? t.kt : t.kb), L, (p == 0 ? t.lt : t.lb), s.nx, n, r, a.b, a.Uc, xl);
                T2 tv; tv.x = (T)(v.x * sc); tv.y = (T)(v.y * sc);
                vecs[p * n + r] = tv;
            }
        }
        __syncthreads();
        // rows held in registers
#pragma unroll
        for (int u = 0; u < PR; ++u) {
            const int e = entry(t, wave + NW * u);
            if (e < 0) continue;
            const int p = e >> 16, r = e & 0xFFFF;
            const T2 *vec = vecs + p * n;
            A ar = 0, ai = 0;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                int col = c * 64 + lane;
                T2 v;
                if (col < n) v = vec[col];
                else { v.x = 0; v.y = 0; }
                ar += m[u][c].x * v.x - m[u][c].y * v.y;
                ai += m[u][c].x * v.y + m[u][c].y * v.x;
            }
            finish_row(line_of(t, p), r, tw_backward((p == 0 ? t.kt : t.kb)), ar, ai);
        }
        // further rows streamed, UN chunks in flight at a time
        constexpr int UN = NCH < 8 ? NCH : 8;
        for (int rho = wave + NW * PR;; rho += NW) {
            const int e = entry(t, rho);
            if (e < 0) break;
            const int p = e >> 16, r = e & 0xFFFF;
            const T2 *vec = vecs + p * n;
            const T2 *row = F + line_of(t, p) * nn + (long)r * n;
            A ar = 0, ai = 0;
            for (int c0 = 0; c0 < NCH; c0 += UN) {
                T2 mm[UN];
#pragma unroll
                for (int c = 0; c < UN; ++c) {
                    int col = (c0 + c) * 64 + lane;
                    if (c0 + c < NCH && col < n) mm[c] = row[col];
                    else { mm[c].x = 0; mm[c].y = 0; }
                }
#pragma unroll
                for (int c = 0; c < UN; ++c) {
                    int col = (c0 + c) * 64 + lane;
                    T2 v;
                    if (c0 + c < NCH && col < n) v = vec[col];
                    else { v.x = 0; v.y = 0; }
                    ar += mm[c].x * v.x - mm[c].y * v.y;
                    ai += mm[c].x * v.y + mm[c].y * v.x;
                }
            }
            finish_row(line_of(t, p), r, tw_backward((p == 0 ? t.kt : t.kb)), ar, ai);
        }
        if (st == S - 1) break;
        // Publish this step, start loading the next one, then wait.  The
        // rows went out as device-coherent stores; once every wave has seen
        // them acknowledged (s_waitcnt before the workgroup barrier) one
        // counter increment publishes them, and readers fetch them with
        // device-coherent loads, so no cache-wide fence is needed.
        __builtin_amdgcn_s_waitcnt(0);   // only this wave's row stores are outstanding
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
        const unsigned target = (unsigned)(st + 1) * team;
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = tw_step(s.nx, st + 1);
        prefetch(t);
        prefetch_o(t);
        if (threadIdx.x == 0) {
            unsigned spins = 0;
            while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > SPIN_LIMIT ||
                    __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
        if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    }
}

// ---------------------------------------------------------------- half storage
// The stored inverses are complex symmetric, so only their upper triangles
// need to be read: y = F v has y_r = sum_{c >= r} F[r][c] v_c (row part) +
// sum_{c < r} F[c][r] v_c (the column parts of the rows above).  Member w of
// a strip's team owns the rows w, w + team, ... of both products, so every
// member streams about the same number of rows and of upper-triangle
// elements; a wave forms the row dot of each of its rows and accumulates
// the rows' column contributions F[r][c] v_r per lane in registers; both go
// into the workgroup's LDS partial (LDS atomics, the column sums once per
// product), which the workgroup publishes for columns c >= w.  After the team barrier every member sums the members'
// partials in member order, finishes the lines (scaling, or the backward
// subtraction from the forward result), keeps them in LDS for its next
// vector phase and stores its own rows to x.  Partials are double-buffered
// by step parity, so a member writing step s + 1 never meets a slower member
// still reading step s.

__device__ __forceinline__ void st_agent2(double2 *p, double2 v) { st_agent(p, v); }
__device__ __forceinline__ double2 ld_agent2(const double2 *p) { return ld_agent(p); }
__device__ __forceinline__ void st_agent2(float2 *p, float2 v) {
    unsigned long long u;
    __builtin_memcpy(&u, &v, sizeof(u));
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float2 ld_agent2(const float2 *p) {
    unsigned long long u = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    float2 v;
    __builtin_memcpy(&v, &u, sizeof(v));
    return v;
}

// Loads through a buffer resource (base, byte range): an offset outside the
// range returns zeros without a memory access (the hardware's range check of
// raw buffers, dword 3 of the resource as on every gfx9 chip).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_range(const void *base, int bytes) {
    // base and range are the same in every lane: the resource lives in
    // scalar registers, stated explicitly for the compiler
    const unsigned long long b = reinterpret_cast<unsigned long long>(base);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    void *p = reinterpret_cast<void *>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, __builtin_amdgcn_readfirstlane(bytes),
                                             0x00020000);
}
__device__ __forceinline__ void range_load(float2 &d, __amdgpu_buffer_rsrc_t rs, unsigned off) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    d.x = __uint_as_float(v.x);
    d.y = __uint_as_float(v.y);
}
__device__ __forceinline__ void range_load(double2 &d, __amdgpu_buffer_rsrc_t rs, unsigned off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    __builtin_memcpy(&d, &v, sizeof(d));
}

__device__ __forceinline__ float fma_acc(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_acc(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Per-wave partial regions in LDS: when NW regions of both products fit
// (with the product vectors and the finished lines) in 120 KiB, each wave
// writes its own column sums with plain stores and the workgroup adds the
// regions in wave order; otherwise the waves add into one partial with LDS
// atomics.  The bound uses the instance's widest line, NCH * 64.
template <typename T, int NW, int NCH>
constexpr bool sym_wave_regions() {
    return (size_t)(NW + 1) * 2 * NCH * 64 * 2 * sizeof(typename acc_t<T>::type) +
               (size_t)2 * NCH * 64 * 2 * sizeof(T) + (size_t)2 * NCH * 64 * 16 <=
           (size_t)120 * 1024;
}

template <typename T, int NW, int NCH, int PR, int SPLIT>
__global__ __launch_bounds__(NW * 64) void strip_solve_sym_kernel(SolveArgs a) {
    typedef typename cplx_of<T>::type T2;
    typedef typename acc_t<T>::type A;
    typedef typename cplx_of<A>::type A2;
    constexpr bool WR = sym_wave_regions<T, NW, NCH>();
    if (solve_skipped(a)) return;
    constexpr int NTHR = NW * 64;
    const int n = a.n;
    // LDS: the kernel has no static LDS, so the dynamic block starts at 0 and
    // every array is aligned to its element (the 64-bit LDS atomics need
    // it); the partial comes first: either NW per-wave regions [NW][2][n]
    // of complex column sums (and, after the other arrays, the rows' own
    // results [2][n]), or one atomically updated [2][n] real and [2][n]
    // imaginary partial that takes both
    extern __shared__ unsigned char smem_raw[];
    A2 *wreg = reinterpret_cast<A2 *>(smem_raw);
    A *pre = reinterpret_cast<A *>(smem_raw);
    A *pim = pre + 2 * n;
    T2 *vecs = WR ? reinterpret_cast<T2 *>(wreg + (size_t)NW * 2 * n)
                  : reinterpret_cast<T2 *>(pim + 2 * n);         // [2][n] product vectors
    double2 *red = reinterpret_cast<double2 *>(vecs + 2 * n);    // [2][n] lines finished last step
    A2 *rres = reinterpret_cast<A2 *>(red + 2 * n);              // [2][n] row results (WR)
    const int nst = a.nstrips, team = a.team;
    const int j = blockIdx.x % nst, w = blockIdx.x / nst;
    const StripMeta s = a.strips[j];
    // member w owns the rows w, w + team, w + 2 team, ...: every member gets
    // long and short rows alike, so row counts and element counts balance
    const int R = w < n ? (n - w + team - 1) / team : 0;
    // the wave index is uniform across the wave: in an SGPR, every per-row
    // quantity derived from it (row, product, chunk range) stays scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const T2 *F = reinterpret_cast<const T2 *>(a.F);
    T2 *parts = reinterpret_cast<T2 *>(a.part) + (long)j * 2 * SOLVE_MAX_TEAM * 2 * n;
    unsigned *ctr = a.counters + j;
    const long nn = (long)n * n;
    const int S = tw_steps(s.nx);
    const double sc = strip_scale(a.lmax ? a.lmax + s.off : nullptr, s.nx), inv = 1.0 / sc;
    // The waves form NG groups of SPLIT: the waves of a group share their
    // rows, wave h of the group taking the chunks c = jj SPLIT + h of each
    // (interleaved, so that the halves of the triangle balance), which
    // divides the registers a row, the vector and the column sums need by
    // SPLIT.  A group's rows k = 0, 1, ... of a step go in groups of PR: the
    // loads of a whole group are issued together, PR rows in flight, and
    // its rows are then multiplied in order as their chunks arrive.  A row
    // is loaded through a buffer resource whose range is its upper part
    // [r, n): the lanes left of the diagonal and past the end of the line
    // get zeros from the range check, without a memory access, and a row
    // past the end of the list has an empty range.  Every group thus issues
    // exactly PR * NCW loads with no branch and no mask.
    constexpr int NG = NW / SPLIT, NCW = (NCH + SPLIT - 1) / SPLIT;
    static_assert(NW % SPLIT == 0, "waves must form whole groups");
    const int h = wave % SPLIT, grp = wave / SPLIT;
    T2 m[PR][NCW], dg[PR];

    auto entry = [&](const TwStep &t, int rho) -> int {
        if (t.lt >= 0) {
            if (rho < R) return w + team * rho;
            rho -= R;
        }
        if (t.lb >= 0 && rho < R) return 65536 + w + team * rho;
        return -1;
    };
    auto line_of = [&](const TwStep &t, int p) -> long { return s.off + (p == 0 ? t.lt : t.lb); };
    auto kind_of = [&](const TwStep &t, int p) -> int { return p == 0 ? t.kt : t.kb; };
    auto own = [&](int c) -> bool { return c % team == w; };
    auto has = [&](const TwStep &t, int p) -> bool { return (p == 0 ? t.lt : t.lb) >= 0; };
    // The per-chunk quantities (column index, clamps, masks, LDS addresses)
    // are cheap to recompute but invariant across rows; the lane index and n
    // pass through an empty asm once per group so that they are recomputed
    // there instead of being hoisted out of the row loop, where 2 x NCH of
    // them would stay live next to the row buffers.
    auto opaque_v = [](int v) { asm volatile("" : "+v"(v)); return v; };
    auto opaque_s = [](int v) { asm volatile("" : "+s"(v)); return v; };
    // rows k .. k + PR - 1 of the wave's list, those from k1 on not wanted
    auto load_group = [&](const TwStep &t, int k, int k1, T2 (&m)[PR][NCW], T2 (&dg)[PR]) {
        const int lane_ = opaque_v(lane) + 64 * h;
#pragma unroll
        for (int u = 0; u < PR; ++u) {
            const int e = k + u < k1 ? entry(t, grp + NG * (k + u)) : -1;
            const bool ok = e >= 0;
            const int p = e >> 16, r = ok ? e & 0xFFFF : 0;
            const T2 *D = ok ? F + line_of(t, p) * nn + (long)r * n + r : F;
            const __amdgpu_buffer_rsrc_t rs = row_range(D, ok ? (n - r) * (int)sizeof(T2) : 0);
            dg[u] = *D;                                 // the diagonal element (uniform)
            // byte offset of column c * 64 + lane from the diagonal: negative
            // offsets wrap past the range
#pragma unroll
            for (int jj = 0; jj < NCW; ++jj)
                range_load(m[u][jj], rs, (unsigned)(jj * SPLIT * 64 + lane_ - r) * (unsigned)sizeof(T2));
        }
    };
    // the wave's first rows of a step (its product from above, else from
    // below), loaded before the team barrier
    auto prefetch = [&](const TwStep &t) { load_group(t, 0, 0x7FFFFFFF, m, dg); };

    // Backward lines overwrite the forward result that every member reads
    // while finishing them, so their rows go to x one barrier later, from
    // red, before red is reused (forward lines are stored at once).  The
    // thread that stores red[c] is the one that overwrites it next.
    auto store_backward = [&](const TwStep &tr) {
        for (int p = 0; p < 2; ++p) {
            if (!has(tr, p) || !tw_backward(kind_of(tr, p))) continue;
            const long L = line_of(tr, p);
            for (int c = threadIdx.x; c < n; c += NTHR)
                if (own(c)) st_agent(a.x + L * n + c, red[p * n + c]);
        }
    };
    auto team_wait = [&](unsigned target) {
        if (threadIdx.x == 0) {
            unsigned spins = 0;
            while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > SPIN_LIMIT ||
                    __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
    };

    TwStep t = tw_step(s.nx, 0), tp = t, tr = t;
    bool red_valid = false;
    prefetch(t);
    for (int st = 0; st <= S; ++st) {
        if (st > 0) {
            if (red_valid) store_backward(tr);   // the lines of step st - 2
            // finish the previous step's lines from the members' partials
            // members u <= c (first row u) hold a partial for column c; the
            // loads of both products go out together in batches of members
            // (after the forward result a backward line subtracts from) and
            // are summed in member order
            const T2 *pb = parts + (long)((st - 1) & 1) * SOLVE_MAX_TEAM * 2 * n;
            for (int c = threadIdx.x; c < n; c += NTHR) {
                const int mc = min(team, c + 1);
                const bool h0 = has(tp, 0), h1 = has(tp, 1);
                double2 o[2];
                A yr[2] = {0, 0}, yi[2] = {0, 0};
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const bool hp = p == 0 ? h0 : h1;
                    o[p] = hp && tw_backward(kind_of(tp, p)) ? ld_agent(a.x + line_of(tp, p) * n + c)
                                                             : cd(0.0, 0.0);
                }
                // (4 members per batch in the 16-wave tiles, whose waves
                // have half the registers)
                constexpr int UB = NW >= 16 ? (sizeof(T) == 8 ? 2 : 4) : 8;
                for (int u0 = 0; u0 < mc; u0 += UB) {
                    T2 v[2][UB];
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int q = 0; q < UB; ++q) {
                            const bool hp = p == 0 ? h0 : h1;
                            if (hp && u0 + q < mc) v[p][q] = ld_agent2(pb + ((long)(u0 + q) * 2 + p) * n + c);
                            else { v[p][q].x = 0; v[p][q].y = 0; }
                        }
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int q = 0; q < UB; ++q) { yr[p] += v[p][q].x; yi[p] += v[p][q].y; }
                }
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    if (!(p == 0 ? h0 : h1)) continue;
                    const long L = line_of(tp, p);
                    double2 xv = cd((double)yr[p] * inv, (double)yi[p] * inv);
                    if (tw_backward(kind_of(tp, p))) {
                        xv = cd(o[p].x - xv.x, o[p].y - xv.y);
                    } else if (own(c)) {
                        st_agent(a.x + L * n + c, xv);
                    }
                    red[p * n + c] = xv;
                }
            }
            tr = tp;
            red_valid = true;
        }
        if (st == S) break;
        __syncthreads();
        // vector phase; lines finished last step come from LDS
        auto xl = [&](long line, int q) -> double2 {
            if (st > 0) {
                if (has(tp, 0) && line == line_of(tp, 0)) return red[q];
                if (has(tp, 1) && line == line_of(tp, 1)) return red[n + q];
            }
            return ld_agent(a.x + line * n + q);
        };
        for (int p = 0; p < 2; ++p) {
            if (!has(t, p)) continue;
            const long L = line_of(t, p);
            for (int r = threadIdx.x; r < n; r += NTHR) {
                double2 v = tw_vec(kind_of(t, p), L, (p == 0 ? t.lt : t.lb), s.nx, n, r, a.b, a.Uc, xl);
                T2 tv; tv.x = (T)(v.x * sc); tv.y = (T)(v.y * sc);
                vecs[p * n + r] = tv;
            }
        }
        if constexpr (!WR)
            for (int i = threadIdx.x; i < 4 * n; i += NTHR) pre[i] = 0;
        else
            for (int i = threadIdx.x; i < 2 * n; i += NTHR) {
                A2 z;
                z.x = 0;
                z.y = 0;
                rres[i] = z;
            }
        __syncthreads();
        // row phase: each row's dot goes to the partial (its own column);
        // its column contributions F[r][c] v_r (c > r) accumulate per lane in
        // registers over the wave's rows of a product and are added to the
        // partial once per product
        A cr[NCW], ci[NCW];
#pragma unroll
        for (int c = 0; c < NCW; ++c) { cr[c] = 0; ci[c] = 0; }
        int flushed = 0;
        auto flush = [&](int p) {
            const int lane_ = opaque_v(lane) + 64 * h, n_ = opaque_s(n);
            if constexpr (WR) {
                A2 *q = wreg + (size_t)(wave * 2 + p) * n;
#pragma unroll
                for (int c = 0; c < NCW; ++c) {
                    const int col = c * SPLIT * 64 + lane_;
                    if (col < n_) {
                        A2 v;
                        v.x = cr[c];
                        v.y = ci[c];
                        q[col] = v;
                    }
                    cr[c] = 0;
                    ci[c] = 0;
                }
            } else {
                A *qre = pre + p * n, *qim = pim + p * n;
#pragma unroll
                for (int c = 0; c < NCW; ++c) {
                    const int col = c * SPLIT * 64 + lane_;
                    if (col < n_) {
                        atomicAdd(&qre[col], cr[c]);
                        atomicAdd(&qim[col], ci[c]);
                    }
                    cr[c] = 0;
                    ci[c] = 0;
                }
            }
            flushed |= 1 << p;
        };
        // the product's vector, chunk c of it in lane order, is the same for
        // every row of the product: held in registers, one LDS read per
        // chunk and product
        T2 vv[NCW];
        auto load_vec = [&](int p) {
            const int lane_ = opaque_v(lane) + 64 * h, n_ = opaque_s(n);
            const T2 *vec = vecs + p * n;
#pragma unroll
            for (int c = 0; c < NCW; ++c) vv[c] = vec[min(c * SPLIT * 64 + lane_, n_ - 1)];
        };
        // A row adds its dot to column r and F[r][c] v_r to every column
        // c >= r; the diagonal term, in both, is taken out of the first once.
        // The arithmetic is 8 fused multiply-adds per chunk (two chains per
        // component of the dot), and a chunk wholly left of the diagonal
        // (zeros from the range check) is skipped by a uniform branch: its
        // load is older than the row's later chunks, so it has completed
        // once they are waited for, and nothing waits for it.
        auto row = [&](int k, const T2 (&mm)[NCW], const T2 &d) {
            const int e = entry(t, grp + NG * k);
            const int p = e >> 16, r = e & 0xFFFF;
            const T2 vr = vecs[p * n + r];
            const A vrx = (A)vr.x, vry = (A)vr.y;
            // two chains where registers allow (16-wave tiles have half)
            constexpr int NCHAIN = NW >= 16 ? 1 : 2;
            A dr[2] = {0, 0}, di[2] = {0, 0};
#pragma unroll
            for (int c = 0; c < NCW; ++c) {
                if ((c * SPLIT + SPLIT - 1) * 64 + 63 < r) continue;
                const A mx = (A)mm[c].x, my = (A)mm[c].y;
                const A vx = (A)vv[c].x, vy = (A)vv[c].y;
                const int q = c % NCHAIN;
                dr[q] = fma_acc(mx, vx, dr[q]);
                dr[q] = fma_acc(-my, vy, dr[q]);
                di[q] = fma_acc(mx, vy, di[q]);
                di[q] = fma_acc(my, vx, di[q]);
                cr[c] = fma_acc(mx, vrx, cr[c]);
                cr[c] = fma_acc(-my, vry, cr[c]);
                ci[c] = fma_acc(mx, vry, ci[c]);
                ci[c] = fma_acc(my, vrx, ci[c]);
            }
            A dre = wave_sum(dr[0] + dr[1]);
            A die = wave_sum(di[0] + di[1]);
            if (lane == 0) {
                // the group's first wave takes the diagonal out
                const A gx = h == 0 ? (A)d.x * (A)vr.x - (A)d.y * (A)vr.y : (A)0;
                const A gy = h == 0 ? (A)d.x * (A)vr.y + (A)d.y * (A)vr.x : (A)0;
                if constexpr (WR && SPLIT == 1) {
                    // row r belongs to one wave of one member: a plain store
                    A2 q;
                    q.x = dre - gx;
                    q.y = die - gy;
                    rres[p * n + r] = q;
                } else if constexpr (WR) {
                    atomicAdd(&rres[p * n + r].x, dre - gx);
                    atomicAdd(&rres[p * n + r].y, die - gy);
                } else {
                    atomicAdd(&pre[p * n + r], dre - gx);
                    atomicAdd(&pim[p * n + r], die - gy);
                }
            }
        };
        // this wave group's rows of the step: k < K0 in the product from above
        const int R0 = has(t, 0) ? R : 0, Rt = R0 + (has(t, 1) ? R : 0);
        const int K0 = R0 > grp ? (R0 - grp + NG - 1) / NG : 0;
        const int Kt = Rt > grp ? (Rt - grp + NG - 1) / NG : 0;
        // one loop per product: rows k0 .. k1 - 1 in groups of PR, the first
        // group already loaded when it was prefetched
        auto run = [&](int p, int k0, int k1, bool first_loaded) {
            load_vec(p);
            for (int k = k0; k < k1; k += PR) {
                if (k > k0 || !first_loaded) load_group(t, k, k1, m, dg);
#pragma unroll
                for (int u = 0; u < PR; ++u)
                    if (k + u < k1) row(k + u, m[u], dg[u]);
            }
            flush(p);
        };
        if (K0 > 0) run(0, 0, K0, true);
        if (Kt > K0) run(1, K0, Kt, K0 == 0);
        if constexpr (WR) {
            // a product this wave had no rows of gets a zero region
            for (int p = 0; p < 2; ++p) {
                if (!has(t, p) || (flushed >> p & 1)) continue;
                A2 *q = wreg + (size_t)(wave * 2 + p) * n;
                A2 z;
                z.x = 0;
                z.y = 0;
                for (int col = lane; col < n; col += 64) q[col] = z;
            }
        }
        __syncthreads();
        // publish this member's partial (columns >= w) for this step
        {
            T2 *pw = parts + (long)(st & 1) * SOLVE_MAX_TEAM * 2 * n + (long)w * 2 * n;
            for (int p = 0; p < 2; ++p) {
                if (!has(t, p)) continue;
                for (int c = w + threadIdx.x; c < n; c += NTHR) {
                    T2 v;
                    if constexpr (WR) {
                        // column c's sums are in the regions of the waves
                        // that take its chunk
                        A sr = 0, si = 0;
                        const int hc = (c >> 6) % SPLIT;
#pragma unroll
                        for (int u = 0; u < NW; u += SPLIT) {
                            const A2 q = wreg[(size_t)((u + hc) * 2 + p) * n + c];
                            sr += q.x;
                            si += q.y;
                        }
                        const A2 q = rres[p * n + c];
                        v.x = (T)(sr + q.x);
                        v.y = (T)(si + q.y);
                    } else {
                        v.x = (T)pre[p * n + c];
                        v.y = (T)pim[p * n + c];
                    }
                    st_agent2(pw + (long)p * n + c, v);
                }
            }
        }
        // team barrier; the next step's rows are loaded while waiting
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
        const unsigned target = (unsigned)(st + 1) * team;
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tp = t;
        if (st + 1 < S) {
            t = tw_step(s.nx, st + 1);
            prefetch(t);
        }
        team_wait(target);
        if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    }
    // the last backward lines: once every member has finished them
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    team_wait((unsigned)(S + 1) * team);
    if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    store_backward(tr);
}

// Batched solve over many strips of different widths and instances.  A
// persistent grid takes work items from a queue (one atomic per item); an
// item is one member of the team of workgroups that solves one strip, the
// members of a strip being consecutive items, and the items of multi-member
// strips coming first so that every team is complete among the first
// workgroups to start.  A member owns the rows [r0, r1) of every product of
// its strip; wave w streams rows r0 + w, r0 + w + NW, ..., RU rows and UN
// column chunks of 64 in flight at a time.  Teams of one synchronise with the
// workgroup barrier only; larger teams add the strip's counter barrier with
// device-coherent row exchange and a bounded wait.
template <typename T, int NW, int RU, int UN>
__global__ __launch_bounds__(NW * 64) void batch_solve_kernel(BatchSolveArgs a) {
    typedef typename cplx_of<T>::type T2;
    typedef typename acc_t<T>::type A;
    extern __shared__ unsigned char smem_raw[];
    T2 *vec = reinterpret_cast<T2 *>(smem_raw);
    __shared__ int item_sh, err_sh;
    constexpr int NTHR = NW * 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned *queue = a.counters + a.nstrips;
    const int nitems = *a.nitems;
    while (true) {
        if (threadIdx.x == 0) {
            int e = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            item_sh = e ? nitems : (int)atomicAdd(queue, 1u);
        }
        __syncthreads();
        const int it = item_sh;
        __syncthreads();
        if (it >= nitems) return;
        const BItem I = a.items[it];
        const BStrip s = a.strips[I.strip];
        if (a.guard && s.ctl && fp_idle(s.ctl)) continue;
        if (a.ran && threadIdx.x == 0) *a.ran = 1;
        const int n = s.n, nx = s.nx, team = I.team;
        const int rpw = (n + team - 1) / team;
        const int r0 = min(n, I.member * rpw), r1 = min(n, r0 + rpw);
        if (a.work && threadIdx.x == 0) {
            // stored inverses: this member's rows of every product; member 0
            // also counts b, x and the coupling coefficients of the strip
            unsigned long long w = (unsigned long long)(2 * nx - 1) * (r1 - r0) * n * sizeof(T2);
            if (I.member == 0) w += (unsigned long long)nx * n * 80;
            atomicAdd(a.work, w);
        }
        const T2 *F = reinterpret_cast<const T2 *>(s.F);
        const long nn = (long)n * n;
        unsigned *ctr = a.counters + I.strip;
        const double sc = strip_scale(s.lmax, nx), inv = 1.0 / sc;
        const int S = tw_steps(nx);
        auto xl = [&](long line, int q) -> double2 { return ld_agent(s.x + line * n + q); };
        for (int k = 0; k < S; ++k) {
            const TwStep t = tw_step(nx, k);
            
            // vector phase: the vectors of both products of this step
            for (int p = 0; p < 2; ++p) {
                if ((p == 0 ? t.lt : t.lb) < 0) continue;
                for (int r = threadIdx.x; r < n; r += NTHR) {
                    double2 v = tw_vec((p == 0 ? t.kt : t.kb), (p == 0 ? t.lt : t.lb), (p == 0 ? t.lt : t.lb), nx, n, r, s.b, s.Uc, xl);
                    T2 tv; tv.x = (T)(v.x * sc); tv.y = (T)(v.y * sc);
                    vec[p * n + r] = tv;
                }
            }
            __syncthreads();
            for (int p = 0; p < 2; ++p) {
                if ((p == 0 ? t.lt : t.lb) < 0) continue;
                const int i = (p == 0 ? t.lt : t.lb);
                const bool bwd = tw_backward((p == 0 ? t.kt : t.kb));
                const T2 *M = F + (long)i * nn;
                const T2 *vp = vec + p * n;
                for (int rb = r0 + wave; rb < r1; rb += NW * RU) {
                    A ar[RU], ai[RU];
                    // forward results of backward rows, loaded ahead of the
                    // products so their latency overlaps them
                    double2 o[RU];
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        ar[u] = 0;
                        ai[u] = 0;
                        const int r = rb + NW * u;
                        o[u] = bwd && r < r1 ? ld_agent(s.x + (long)i * n + r) : cd(0.0, 0.0);
                    }
                    for (int c0 = 0; c0 < n; c0 += 64 * UN) {
                        T2 mm[RU][UN];
#pragma unroll
                        for (int u = 0; u < RU; ++u)
#pragma unroll
                            for (int kk = 0; kk < UN; ++kk) {
                                int r = rb + NW * u, c = c0 + lane + 64 * kk;
                                if (r < r1 && c < n) mm[u][kk] = M[(long)r * n + c];
                                else { mm[u][kk].x = 0; mm[u][kk].y = 0; }
                            }
#pragma unroll
                        for (int kk = 0; kk < UN; ++kk) {
                            int c = c0 + lane + 64 * kk;
                            T2 v;
                            if (c < n) v = vp[c];
                            else { v.x = 0; v.y = 0; }
#pragma unroll
                            for (int u = 0; u < RU; ++u) {
                                ar[u] += mm[u][kk].x * v.x - mm[u][kk].y * v.y;
                                ai[u] += mm[u][kk].x * v.y + mm[u][kk].y * v.x;
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        A sr = wave_sum(ar[u]);
                        A si = wave_sum(ai[u]);
                        int r = rb + NW * u;
                        if (lane == 0 && r < r1) {
                            double2 *xr = s.x + (long)i * n + r;
                            if (!bwd) st_agent(xr, cd((double)sr * inv, (double)si * inv));
                            else st_agent(xr, cd(o[u].x - (double)sr * inv, o[u].y - (double)si * inv));
                        }
                    }
                }
            }
            if (k == S - 1) break;
            // publish this step: stores acknowledged, workgroup barrier,
            // and for a team the strip counter
            __builtin_amdgcn_s_waitcnt(0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __syncthreads();
            if (team > 1) {
                if (threadIdx.x == 0) {
                    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const unsigned target = (unsigned)(k + 1) * team;
                    unsigned spins = 0;
                    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                           target) {
                        __builtin_amdgcn_s_sleep(2);
                        if (++spins > SPIN_LIMIT ||
                            __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            break;
                        }
                    }
                    err_sh = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __syncthreads();
                if (err_sh) return;
            }
        }
        __syncthreads();
    }
}

__global__ void zero_u32_kernel(unsigned *p, int n, int *err, int *ran) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
    if (i == 0) {
        if (err) *err = 0;
        if (ran) *ran = 0;
    }
}


// Kernel variant for a column count n and a precision: the prefetching
// kernel with a register tile sized to stay under the VGPR budget, or the
// generic kernel beyond 33 column chunks.
struct Variant {
    const void *fn;
    int threads;
    int wregs;   // upper-triangle kernel with per-wave partial regions
    int ofwd;    // full-row kernel staging backward rows' forward results in LDS
};

// Tile shapes of the strip solve for a column count n and a precision: the
// prefetching kernel with NW waves and PR rows in registers per wave (lighter
// shapes fit two workgroups per CU, and so larger teams), or the generic
// kernel beyond 33 column chunks.  The autotuner times every shape with
// every feasible team size.
constexpr int SOLVE_SHAPES = 4;

Variant variant_for(int n, int fp32, int shape = 0) {
    int nch = (n + 63) / 64;
    shape = shape < 0 ? 0 : (shape >= SOLVE_SHAPES ? SOLVE_SHAPES - 1 : shape);
    if (fp32) {
        if (nch <= 3) {
            if (shape == 0) return {(const void *)strip_solve_pf_kernel<float, 8, 3, 8>, 512, 0, 1};
            if (shape == 1) return {(const void *)strip_solve_pf_kernel<float, 8, 3, 3>, 512, 0, 1};
            return {(const void *)strip_solve_pf_kernel<float, 16, 3, 2>, 1024, 0, 1};
        }
        if (nch <= 9) {
            if (shape == 0) return {(const void *)strip_solve_pf_kernel<float, 8, 9, 5>, 512, 0, 1};
            if (shape == 1) return {(const void *)strip_solve_pf_kernel<float, 8, 9, 2>, 512, 0, 1};
            if (shape == 2) return {(const void *)strip_solve_pf_kernel<float, 16, 9, 2>, 1024, 0, 1};
            return {(const void *)strip_solve_pf_kernel<float, 8, 9, 9>, 512, 0, 1};
        }
        if (nch <= 17) {
            if (shape == 0) return {(const void *)strip_solve_pf_kernel<float, 8, 17, 3>, 512, 0, 1};
            if (shape == 1) return {(const void *)strip_solve_pf_kernel<float, 8, 17, 1>, 512, 0, 1};
            if (shape == 2) return {(const void *)strip_solve_pf_kernel<float, 16, 17, 1>, 1024, 0, 1};
            return {(const void *)strip_solve_pf_kernel<float, 8, 17, 4>, 512, 0, 1};
        }
        if (nch <= 33) return {(const void *)strip_solve_pf_kernel<float, 8, 33, 1>, 512, 0, 1};
        return {(const void *)strip_solve_kernel<float>, SOLVE_THREADS};
    }
    if (nch <= 3) {
        if (shape == 1) return {(const void *)strip_solve_pf_kernel<double, 8, 3, 4>, 512, 0, 1};
        return {(const void *)strip_solve_pf_kernel<double, 16, 3, 4>, 1024, 0, 1};
    }
    if (nch <= 9) {
        if (shape == 0) return {(const void *)strip_solve_pf_kernel<double, 8, 9, 3>, 512, 0, 1};
        if (shape == 1) return {(const void *)strip_solve_pf_kernel<double, 8, 9, 1>, 512, 0, 1};
        if (shape == 2) return {(const void *)strip_solve_pf_kernel<double, 16, 9, 1>, 1024, 0, 1};
        return {(const void *)strip_solve_pf_kernel<double, 8, 9, 4>, 512, 0, 1};
    }
    if (nch <= 17) return {(const void *)strip_solve_pf_kernel<double, 8, 17, 1>, 512, 0, 1};
    return {(const void *)strip_solve_kernel<double>, SOLVE_THREADS};
}

// Half-storage kernels, same tile shapes; null beyond 33 (c32) or 17 (FP64)
// column chunks.
Variant variant_sym_for(int n, int fp32, int shape) {
    int nch = (n + 63) / 64;
    shape = shape < 0 ? 0 : (shape >= SOLVE_SHAPES ? SOLVE_SHAPES - 1 : shape);
    if (fp32) {
        if (nch <= 3) {
            if (shape == 0) return {(const void *)strip_solve_sym_kernel<float, 8, 3, 8, 1>, 512,
                    (int)sym_wave_regions<float, 8, 3>()};
            if (shape == 1) return {(const void *)strip_solve_sym_kernel<float, 8, 3, 3, 1>, 512,
                    (int)sym_wave_regions<float, 8, 3>()};
            return {(const void *)strip_solve_sym_kernel<float, 16, 3, 2, 1>, 1024,
                    (int)sym_wave_regions<float, 16, 3>()};
        }
        if (nch <= 9) {
            if (shape == 0) return {(const void *)strip_solve_sym_kernel<float, 8, 9, 5, 1>, 512,
                    (int)sym_wave_regions<float, 8, 9>()};
            if (shape == 1) return {(const void *)strip_solve_sym_kernel<float, 8, 9, 2, 1>, 512,
                    (int)sym_wave_regions<float, 8, 9>()};
            if (shape == 2) return {(const void *)strip_solve_sym_kernel<float, 16, 9, 2, 1>, 1024,
                    (int)sym_wave_regions<float, 16, 9>()};
            return {(const void *)strip_solve_sym_kernel<float, 8, 9, 3, 1>, 512,
                    (int)sym_wave_regions<float, 8, 9>()};
        }
        if (nch <= 17) {
            if (shape == 0) return {(const void *)strip_solve_sym_kernel<float, 8, 17, 2, 1>, 512,
                    (int)sym_wave_regions<float, 8, 17>()};
            if (shape == 1) return {(const void *)strip_solve_sym_kernel<float, 8, 17, 1, 1>, 512,
                    (int)sym_wave_regions<float, 8, 17>()};
            if (shape == 2) return {(const void *)strip_solve_sym_kernel<float, 4, 17, 4, 1>, 256,
                    (int)sym_wave_regions<float, 4, 17>()};
            return {(const void *)strip_solve_sym_kernel<float, 4, 17, 3, 1>, 256,
                    (int)sym_wave_regions<float, 4, 17>()};
        }
        if (nch <= 33) {
            // one workgroup per CU (the LDS of ny ~ 2049): rows in flight per
            // CU = waves x rows per group
            if (shape == 0) return {(const void *)strip_solve_sym_kernel<float, 8, 33, 1, 1>, 512,
                    (int)sym_wave_regions<float, 8, 33>()};
            if (shape == 1) return {(const void *)strip_solve_sym_kernel<float, 8, 33, 3, 2>, 512,
                    (int)sym_wave_regions<float, 8, 33>()};
            if (shape == 2) return {(const void *)strip_solve_sym_kernel<float, 8, 33, 4, 2>, 512,
                    (int)sym_wave_regions<float, 8, 33>()};
            return {(const void *)strip_solve_sym_kernel<float, 16, 33, 3, 4>, 1024,
                    (int)sym_wave_regions<float, 16, 33>()};
        }
        return {nullptr, 0};
    }
    if (nch <= 3) {
        if (shape == 1) return {(const void *)strip_solve_sym_kernel<double, 8, 3, 4, 1>, 512,
                    (int)sym_wave_regions<double, 8, 3>()};
        return {(const void *)strip_solve_sym_kernel<double, 16, 3, 2, 1>, 1024,
                    (int)sym_wave_regions<double, 16, 3>()};
    }
    if (nch <= 9) {
        if (shape == 0) return {(const void *)strip_solve_sym_kernel<double, 8, 9, 3, 1>, 512,
                    (int)sym_wave_regions<double, 8, 9>()};
        if (shape == 1) return {(const void *)strip_solve_sym_kernel<double, 8, 9, 1, 1>, 512,
                    (int)sym_wave_regions<double, 8, 9>()};
        if (shape == 2) return {(const void *)strip_solve_sym_kernel<double, 16, 9, 1, 2>, 1024,
                    (int)sym_wave_regions<double, 16, 9>()};
        return {(const void *)strip_solve_sym_kernel<double, 8, 9, 2, 1>, 512,
                    (int)sym_wave_regions<double, 8, 9>()};
    }
    if (nch <= 17) {
        if (shape == 0) return {(const void *)strip_solve_sym_kernel<double, 8, 17, 1, 1>, 512,
                    (int)sym_wave_regions<double, 8, 17>()};
        if (shape == 1) return {(const void *)strip_solve_sym_kernel<double, 8, 17, 2, 2>, 512,
                    (int)sym_wave_regions<double, 8, 17>()};
        if (shape == 2) return {(const void *)strip_solve_sym_kernel<double, 8, 17, 3, 2>, 512,
                    (int)sym_wave_regions<double, 8, 17>()};
        return {(const void *)strip_solve_sym_kernel<double, 16, 17, 1, 4>, 1024,
                    (int)sym_wave_regions<double, 16, 17>()};
    }
    return {nullptr, 0, 0};
}

// dynamic LDS of a strip-solve variant for lines of n nodes
size_t solve_smem(int n, int fp32, int sym, const Variant &v) {
    const size_t e2 = fp32 ? sizeof(float2) : sizeof(double2), ea = fp32 ? 4 : 8;
    if (!sym) return 2 * (size_t)n * e2 + (v.ofwd ? 2 * (size_t)n * sizeof(double2) : 0);
    const size_t rest = 2 * (size_t)n * e2 + 2 * (size_t)n * sizeof(double2);
    if (v.wregs) return (size_t)(v.threads / 64 + 1) * 2 * n * 2 * ea + rest;
    return rest + 4 * (size_t)n * ea;
}

Variant pick(int n, int fp32, int shape, int sym) {
    return sym ? variant_sym_for(n, fp32, shape) : variant_for(n, fp32, shape);
}

}  // namespace

// Shapes 0 .. 3 are the full-row kernels, 4 .. 7 the upper-triangle
// kernels with the same tile (absent beyond their column-chunk limits).
int solve_shapes() { return 2 * SOLVE_SHAPES; }
int solve_shape_is_sym(int shape) { return shape >= SOLVE_SHAPES ? 1 : 0; }

// largest dynamic LDS of the full-row solve's tile shapes (or of the
// generic kernel beyond their column-chunk limit) for lines of n nodes
size_t solve_pf_smem(int n, int fp32) {
    size_t m = 0;
    for (int shape = 0; shape < SOLVE_SHAPES; ++shape)
        m = std::max(m, solve_smem(n, fp32, 0, variant_for(n, fp32, shape)));
    return m;
}

int solve_sym_supported(int n, int fp32) {
    int dev = 0, lim = 0;
    if (!variant_sym_for(n, fp32, 0).fn) return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    for (int shape = 0; shape < SOLVE_SHAPES; ++shape) {
        Variant v = variant_sym_for(n, fp32, shape);
        if (v.fn && solve_smem(n, fp32, 1, v) > (size_t)lim) return 0;
    }
    return 1;
}

int solve_max_resident_blocks(int fp32, int n, int shape) {
    int dev = 0, cus = 0, per = 0;
    const int sym = solve_shape_is_sym(shape);
    if (sym && !solve_sym_supported(n, fp32)) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    Variant v = pick(n, fp32, shape % SOLVE_SHAPES, sym);
    if (!v.fn) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, v.fn, v.threads,
                                                     solve_smem(n, fp32, sym, v)) != hipSuccess)
        return 0;
    return per * cus;
}

hipError_t launch_strip_solve(hipStream_t st, const SolveArgs &a, int fp32, hipEvent_t ev0,
                              hipEvent_t ev1) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3((a.nstrips + 255) / 256), dim3(256), 0, st,
                       a.counters, a.nstrips, (int *)nullptr, a.ran);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SolveArgs args = a;
    void *params[] = {&args};
    const int sym = solve_shape_is_sym(a.shape);
    if (sym && (a.team > SOLVE_MAX_TEAM || !a.part)) return hipErrorInvalidConfiguration;
    Variant v = pick(a.n, fp32, a.shape % SOLVE_SHAPES, sym);
    if (!v.fn) return hipErrorInvalidConfiguration;
    size_t smem = solve_smem(a.n, fp32, sym, v);
    dim3 grid(a.nstrips * a.team), block(v.threads);
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    e = hipLaunchCooperativeKernel(v.fn, grid, block, params, (unsigned)smem, st);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, st);
    return e;
}

// ---------------------------------------------------------------- batched solve
namespace {

struct BVariant {
    const void *fn;
    int threads;
    const char *name;
};

BVariant batch_variant(int fp32, int v) {
    if (fp32) {
        switch (v) {
        case 0: return {(const void *)batch_solve_kernel<float, 8, 2, 8>, 512, "c32 8w ru2 un8"};
        case 1: return {(const void *)batch_solve_kernel<float, 8, 4, 8>, 512, "c32 8w ru4 un8"};
        case 2: return {(const void *)batch_solve_kernel<float, 4, 4, 8>, 256, "c32 4w ru4 un8"};
        default: return {(const void *)batch_solve_kernel<float, 16, 2, 8>, 1024, "c32 16w ru2 un8"};
        }
    }
    switch (v) {
    case 0: return {(const void *)batch_solve_kernel<double, 8, 2, 4>, 512, "c128 8w ru2 un4"};
    case 1: return {(const void *)batch_solve_kernel<double, 8, 4, 4>, 512, "c128 8w ru4 un4"};
    case 2: return {(const void *)batch_solve_kernel<double, 4, 4, 4>, 256, "c128 4w ru4 un4"};
    default: return {(const void *)batch_solve_kernel<double, 16, 2, 4>, 1024, "c128 16w ru2 un4"};
    }
}

}  // namespace

int batch_solve_variants() { return 4; }

const char *batch_solve_variant_name(int fp32, int variant) { return batch_variant(fp32, variant).name; }

int batch_solve_max_resident_blocks(int fp32, int variant, int max_n) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    BVariant v = batch_variant(fp32, variant);
    size_t smem = 2 * (size_t)max_n * (fp32 ? sizeof(float2) : sizeof(double2));
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, v.fn, v.threads, smem) != hipSuccess)
        return 0;
    return per * cus;
}

hipError_t launch_clear_flag(hipStream_t st, int *flag) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, st, (unsigned *)nullptr, 0, flag,
                       (int *)nullptr);
    return hipGetLastError();
}

hipError_t launch_batch_solve(hipStream_t st, const BatchSolveArgs &a, int fp32, int variant,
                              int grid, int max_n, hipEvent_t ev0, hipEvent_t ev1) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3((a.nstrips + 1 + 255) / 256), dim3(256), 0, st,
                       a.counters, a.nstrips + 1, (int *)nullptr, a.ran);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    BVariant v = batch_variant(fp32, variant);
    size_t smem = 2 * (size_t)max_n * (fp32 ? sizeof(float2) : sizeof(double2));
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    BatchSolveArgs args = a;
    void *params[] = {&args};
    e = hipLaunchKernel(v.fn, dim3(grid), dim3(v.threads), params, smem, st);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, st);
    return e;
}
