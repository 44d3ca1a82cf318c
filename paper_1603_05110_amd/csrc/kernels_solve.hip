// Block-tridiagonal substitution with the stored inverses S_i^{-1}:
//   forward   y_i = S_i^{-1} (b_i - U_{i-1}^T y_{i-1}),   i = 0 .. nx-1
//   backward  x_i = y_i - S_i^{-1} (U_i x_{i+1}),          i = nx-2 .. 0
// for every strip at once.  This is the local solve that the fixed point,
// the classical iteration and every outer preconditioned iteration repeat
// (Section 2.2, eq. NproblemRobinNL; Section 5: LU solves of the strip
// systems).  Each step is a dense ny x ny matrix-vector product streamed
// from HBM, so the kernel is bandwidth-bound.
//
// Launch: one persistent cooperative grid, `team` workgroups per strip; the
// workgroup with blockIdx b serves strip b % nstrips (so with a strip count
// that is a multiple of 8 a strip's team sits on one XCD) and owns a
// contiguous row range of every product, spread round-robin over its four
// waves.  Consecutive products of a strip are ordered by a per-strip
// counter barrier: stores drained, one agent-scope release by the arriving
// wave, relaxed polling with backoff, one acquire after the wait.  The wait
// is bounded and sets an error flag, so no wave can spin forever.
#include "osm_internal.h"

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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// out[r] = sum_c M[r][c] vec[c] for rows r in [r0, r1) of one workgroup.
// Wave w takes rows r0 + w, r0 + w + 4, ...; RU of its rows at a time, and
// UN column chunks of 64 per pass, all loads issued before the FMAs.
// mode 0: x[r] = out; mode 1: x[r] -= out.
template <typename T, int RU, int UN>
__device__ __forceinline__ void wg_gemv(const typename cplx_of<T>::type *__restrict__ M, int n,
                                        int r0, int r1, const typename cplx_of<T>::type *vec,
                                        double2 *__restrict__ x, int mode) {
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
                if (mode == 0) x[r] = cd((double)sr, (double)si);
                else {
                    double2 o = x[r];
                    x[r] = cd(o.x - (double)sr, o.y - (double)si);
                }
            }
        }
    }
}

template <typename T> struct tile_shape;
template <> struct tile_shape<float> { static constexpr int RU = 2, UN = 8; };
template <> struct tile_shape<double> { static constexpr int RU = 2, UN = 4; };

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
    T2 *vec = reinterpret_cast<T2 *>(smem_raw);
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
    // forward sweep
    for (int i = 0; i < s.nx; ++i) {
        long L = s.off + i;
        for (int r = threadIdx.x; r < n; r += SOLVE_THREADS) {
            double2 wv = a.b[L * n + r];
            if (i > 0) {
                for (int q = max(r - 1, 0); q <= min(r + 1, n - 1); ++q) {
                    double2 u = a.Uc[((L - 1) * n + q) * 3 + (r - q + 1)];   // U_{i-1}(q, r)
                    wv = csub(wv, cmul(u, a.x[(L - 1) * n + q]));
                }
            }
            T2 t; t.x = (T)wv.x; t.y = (T)wv.y;
            vec[r] = t;
        }
        __syncthreads();
        wg_gemv<T, RU, UN>(F + L * nn, n, r0, r1, vec, a.x + L * n, 0);
        team_barrier(ctr, (++epoch) * team, a.error);
        if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    }
    // backward sweep
    for (int i = s.nx - 2; i >= 0; --i) {
        long L = s.off + i;
        for (int r = threadIdx.x; r < n; r += SOLVE_THREADS) {
            double2 zv = cd(0.0, 0.0);
            for (int q = max(r - 1, 0); q <= min(r + 1, n - 1); ++q) {
                double2 u = a.Uc[(L * n + r) * 3 + (q - r + 1)];             // U_i(r, q)
                zv = cadd(zv, cmul(u, a.x[(L + 1) * n + q]));
            }
            T2 t; t.x = (T)zv.x; t.y = (T)zv.y;
            vec[r] = t;
        }
        __syncthreads();
        wg_gemv<T, RU, UN>(F + L * nn, n, r0, r1, vec, a.x + L * n, 1);
        if (i > 0) {
            team_barrier(ctr, (++epoch) * team, a.error);
            if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
        }
    }
}

// Prefetching variant for ny <= 64 NCH.  Each of the NW waves owns whole
// rows (r0 + wave + NW u) and keeps the first PR of them, NCH column chunks
// of 64, in registers.  Right after the workgroup has published its rows of
// product k and arrived at the strip barrier, it loads its rows of product
// k+1 (the stored inverses do not depend on the vector), so the HBM stream
// overlaps the barrier wait and the next vector phase.
template <typename T, int NW, int NCH, int PR>
__global__ __launch_bounds__(NW * 64) void strip_solve_pf_kernel(SolveArgs a) {
    typedef typename cplx_of<T>::type T2;
    typedef typename acc_t<T>::type A;
    if (solve_skipped(a)) return;
    extern __shared__ unsigned char smem_raw[];
    T2 *vec = reinterpret_cast<T2 *>(smem_raw);
    constexpr int NTHR = NW * 64;
    const int nst = a.nstrips, team = a.team;
    const int j = blockIdx.x % nst, w = blockIdx.x / nst;
    const StripMeta s = a.strips[j];
    const int n = a.n;
    const int rpw = (n + team - 1) / team;
    const int r0 = min(n, w * rpw), r1 = min(n, r0 + rpw);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const T2 *F = reinterpret_cast<const T2 *>(a.F);
    unsigned *ctr = a.counters + j;
    const long nn = (long)n * n;
    const int S = 2 * s.nx - 1;   // forward products i = 0..nx-1, then backward i = nx-2..0
    T2 m[PR][NCH];

    auto line_of = [&](int k) -> long { return s.off + (k < s.nx ? k : 2 * s.nx - 2 - k); };
    auto prefetch = [&](long L) {
        const T2 *M = F + L * nn;
#pragma unroll
        for (int u = 0; u < PR; ++u) {
            int r = r0 + wave + NW * u;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                int col = c * 64 + lane;
                if (r < r1 && col < n) m[u][c] = M[(long)r * n + col];
                else { m[u][c].x = 0; m[u][c].y = 0; }
            }
        }
    };
    auto finish_row = [&](long L, int r, bool fwd, A ar, A ai) {
        ar = wave_sum(ar);
        ai = wave_sum(ai);
        if (lane == 0 && r < r1) {
            double2 *xr = a.x + L * n + r;
            if (fwd) st_agent(xr, cd((double)ar, (double)ai));
            else {
                double2 o = ld_agent(xr);
                st_agent(xr, cd(o.x - (double)ar, o.y - (double)ai));
            }
        }
    };

    prefetch(line_of(0));
    for (int k = 0; k < S; ++k) {
        const long L = line_of(k);
        const bool fwd = k < s.nx;
        const int i = (int)(L - s.off);
        // vector phase: all loads of an entry issued together
        for (int r = threadIdx.x; r < n; r += NTHR) {
            double2 acc = cd(0.0, 0.0);
            double2 cu[3], xv[3];
            if (fwd) {
                acc = a.b[L * n + r];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    int q = r - 1 + d;
                    bool ok = i > 0 && q >= 0 && q < n;
                    // U_{i-1}(q, r)
                    cu[d] = ok ? a.Uc[((L - 1) * n + q) * 3 + (2 - d)] : cd(0.0, 0.0);
                    xv[d] = ok ? ld_agent(a.x + (L - 1) * n + q) : cd(0.0, 0.0);
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) acc = csub(acc, cmul(cu[d], xv[d]));
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    int q = r - 1 + d;
                    bool ok = q >= 0 && q < n;
                    // U_i(r, q)
                    cu[d] = ok ? a.Uc[(L * n + r) * 3 + d] : cd(0.0, 0.0);
                    xv[d] = ok ? ld_agent(a.x + (L + 1) * n + q) : cd(0.0, 0.0);
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) acc = cadd(acc, cmul(cu[d], xv[d]));
            }
            T2 t; t.x = (T)acc.x; t.y = (T)acc.y;
            vec[r] = t;
        }
        __syncthreads();
        // rows held in registers
#pragma unroll
        for (int u = 0; u < PR; ++u) {
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
            finish_row(L, r0 + wave + NW * u, fwd, ar, ai);
        }
        // further rows streamed, UN chunks in flight at a time
        constexpr int UN = NCH < 8 ? NCH : 8;
        for (int r = r0 + wave + NW * PR; r < r1; r += NW) {
            const T2 *row = F + L * nn + (long)r * n;
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
            finish_row(L, r, fwd, ar, ai);
        }
        if (k == S - 1) break;
        // Publish this product, start loading the next one, then wait.  The
        // rows went out as device-coherent stores; once every wave has seen
        // them acknowledged (s_waitcnt before the workgroup barrier) one
        // counter increment publishes them, and readers fetch them with
        // device-coherent loads, so no cache-wide fence is needed.
        __builtin_amdgcn_s_waitcnt(0);   // only this wave's row stores are outstanding
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
        const unsigned target = (unsigned)(k + 1) * team;
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        prefetch(line_of(k + 1));
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

__global__ void zero_u32_kernel(unsigned *p, int n, int *err, int *ran) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
    if (i == 0) {
        *err = 0;
        if (ran) *ran = 0;
    }
}

// Kernel variant for a column count n and a precision: the prefetching
// kernel with a register tile sized to stay under the VGPR budget, or the
// generic kernel beyond 33 column chunks.
struct Variant {
    const void *fn;
    int threads;
};

Variant variant_for(int n, int fp32) {
    int nch = (n + 63) / 64;
    if (fp32) {
        if (nch <= 3) return {(const void *)strip_solve_pf_kernel<float, 8, 3, 8>, 512};
        if (nch <= 9) return {(const void *)strip_solve_pf_kernel<float, 8, 9, 5>, 512};
        if (nch <= 17) return {(const void *)strip_solve_pf_kernel<float, 8, 17, 3>, 512};
        if (nch <= 33) return {(const void *)strip_solve_pf_kernel<float, 8, 33, 1>, 512};
        return {(const void *)strip_solve_kernel<float>, SOLVE_THREADS};
    }
    if (nch <= 3) return {(const void *)strip_solve_pf_kernel<double, 16, 3, 4>, 1024};
    if (nch <= 9) return {(const void *)strip_solve_pf_kernel<double, 8, 9, 3>, 512};
    if (nch <= 17) return {(const void *)strip_solve_pf_kernel<double, 8, 17, 1>, 512};
    return {(const void *)strip_solve_kernel<double>, SOLVE_THREADS};
}

}  // namespace

int solve_max_resident_blocks(int fp32, int n) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    Variant v = variant_for(n, fp32);
    size_t smem = (size_t)n * (fp32 ? sizeof(float2) : sizeof(double2));
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, v.fn, v.threads, smem) != hipSuccess)
        return 0;
    return per * cus;
}

hipError_t launch_strip_solve(hipStream_t st, const SolveArgs &a, int fp32, hipEvent_t ev0,
                              hipEvent_t ev1) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3((a.nstrips + 255) / 256), dim3(256), 0, st,
                       a.counters, a.nstrips, a.error, a.ran);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SolveArgs args = a;
    void *params[] = {&args};
    Variant v = variant_for(a.n, fp32);
    size_t smem = (size_t)a.n * (fp32 ? sizeof(float2) : sizeof(double2));
    dim3 grid(a.nstrips * a.team), block(v.threads);
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    e = hipLaunchCooperativeKernel(v.fn, grid, block, params, (unsigned)smem, st);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, st);
    return e;
}
