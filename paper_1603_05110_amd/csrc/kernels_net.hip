// Learned interface guess: a 1-D convolutional network over the ny nodes of
// every interface line corrects the linear extrapolation 2 g_{n-1} - g_{n-2}
// of the interface vector to the next time step (the paper starts each step
// from the previous converged vector, Section 5; the prediction only moves
// that start, the Schwarz fixed point is unchanged).
//
// Network: conv1d(9 -> 64, kernel 5, zero padding 2) -> GELU (erf form) ->
// conv1d(64 -> 4, kernel 5, zero padding 2), cross-correlation convention.
// Parameters live as an FP32 master copy and a bfloat16 copy (round to
// nearest even); every product uses the bf16 values widened to FP32 and
// accumulates in FP32.  Flat parameter order: W1 (64,9,5), b1 (64),
// W2 (4,64,5), b2 (4).
//
// Kernels: inference over tiles of 64 positions; training with one block per
// trace that walks the trace in tiles, recomputes the halo it needs, and
// accumulates the gradient of the parameters each thread owns in registers
// (no atomics, deterministic); a reduction over traces; Adam.
#include "osm_internal.h"

namespace {

constexpr int CIN = 9, HID = 64, COUT = 4, KW = 5, PAD = 2;
constexpr int NW1 = HID * CIN * KW, NB1 = HID, NW2 = COUT * HID * KW, NB2 = COUT;
constexpr int OW1 = 0, OB1 = NW1, OW2 = NW1 + NB1, OB2 = NW1 + NB1 + NW2;
constexpr int NPAR = NW1 + NB1 + NW2 + NB2;
constexpr int TILE = 64;
constexpr int NT = 256;
constexpr int PPT = (NPAR + NT - 1) / NT;   // parameters owned per thread in training

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__device__ __forceinline__ void load_params(const uint16_t *pbf, float *w) {
    for (int i = threadIdx.x; i < NPAR; i += blockDim.x) w[i] = bf16_to_f32(pbf[i]);
}

// x tile of positions [p0, p0 + n) of trace t (zero outside [0, L)).
__device__ __forceinline__ void load_x(const float *X, int t, int L, int p0, int n, float *xs) {
    for (int e = threadIdx.x; e < CIN * n; e += blockDim.x) {
        int ci = e / n, j = e - ci * n, a = p0 + j;
        xs[e] = (a >= 0 && a < L) ? X[((long)t * CIN + ci) * L + a] : 0.0f;
    }
}

// hidden layer on positions [p0, p0 + nh): z = gelu(h) inside [0, L), 0
// outside (the zero padding of the second convolution); xs holds positions
// [p0 - 2, p0 + nh + 2).  gp (optional) receives gelu'(h) at positions
// [g0, g0 + ng).
__device__ __forceinline__ void hidden(const float *w, const float *xs, int nx, int p0, int nh,
                                       int L, float *zs, float *gp, int g0, int ng) {
    for (int e = threadIdx.x; e < HID * nh; e += blockDim.x) {
        int c = e / nh, j = e - c * nh, a = p0 + j;
        float h = w[OB1 + c];
        const float *wc = w + OW1 + c * CIN * KW;
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
            for (int k = 0; k < KW; ++k) h += wc[ci * KW + k] * xs[ci * nx + j + k];
        bool in = a >= 0 && a < L;
        zs[c * nh + j] = in ? gelu(h) : 0.0f;
        if (gp && a >= g0 && a < g0 + ng) gp[c * ng + (a - g0)] = in ? gelu_grad(h) : 0.0f;
    }
}

// output layer at positions [p0, p0 + ny); zs holds [p0 - 2, p0 + ny + 2).
__device__ __forceinline__ float out_at(const float *w, const float *zs, int nz, int o, int j) {
    float y = w[OB2 + o];
    const float *wo = w + OW2 + o * HID * KW;
    for (int c = 0; c < HID; ++c)
#pragma unroll
        for (int k = 0; k < KW; ++k) y += wo[c * KW + k] * zs[c * nz + j + k];
    return y;
}

__global__ __launch_bounds__(NT) void net_forward_kernel(const uint16_t *pbf, const float *X,
                                                         int L, float *Y) {
    __shared__ float w[NPAR];
    __shared__ float xs[CIN * (TILE + 8)];
    __shared__ float zs[HID * (TILE + 4)];
    const int t = blockIdx.y, a0 = blockIdx.x * TILE;
    load_params(pbf, w);
    load_x(X, t, L, a0 - 4, TILE + 8, xs);
    __syncthreads();
    hidden(w, xs, TILE + 8, a0 - 2, TILE + 4, L, zs, nullptr, 0, 0);
    __syncthreads();
    for (int e = threadIdx.x; e < COUT * TILE; e += blockDim.x) {
        int o = e / TILE, j = e - o * TILE, a = a0 + j;
        if (a < L) Y[((long)t * COUT + o) * L + a] = out_at(w, zs, TILE + 4, o, j);
    }
}

// One block per trace.  Per tile of positions [a0, a0 + 64): hidden layer on
// [a0 - 4, a0 + 68), output and dL/dy on [a0 - 2, a0 + 66), dL/dz and dL/dh
// on the tile; every thread adds the tile's contribution to the gradient of
// the parameters it owns.  dL/dy = 2 (y - target) / (T * 4 * L).
__global__ __launch_bounds__(NT) void net_train_kernel(const uint16_t *pbf, const float *X,
                                                       const float *Yt, int T, int L,
                                                       float *gpart, float *lpart) {
    __shared__ float w[NPAR];
    __shared__ float xs[CIN * (TILE + 12)];
    __shared__ float zs[HID * (TILE + 8)];
    __shared__ float dys[COUT * (TILE + 4)];
    __shared__ float dh[HID * TILE];
    __shared__ float red[NT];
    const int t = blockIdx.x;
    const float inv_n = 2.0f / ((float)T * COUT * (float)L);
    load_params(pbf, w);
    float acc[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) acc[u] = 0.0f;
    float lsum = 0.0f;
    for (int a0 = 0; a0 < L; a0 += TILE) {
        __syncthreads();
        load_x(X, t, L, a0 - 6, TILE + 12, xs);
        __syncthreads();
        hidden(w, xs, TILE + 12, a0 - 4, TILE + 8, L, zs, dh, a0, TILE);
        __syncthreads();
        for (int e = threadIdx.x; e < COUT * (TILE + 4); e += blockDim.x) {
            int o = e / (TILE + 4), j = e - o * (TILE + 4), a = a0 - 2 + j;
            float d = 0.0f;
            if (a >= 0 && a < L) {
                float y = out_at(w, zs, TILE + 8, o, j);
                float r = y - Yt[((long)t * COUT + o) * L + a];
                d = inv_n * r;
                if (j >= 2 && j < TILE + 2) lsum += r * r;
            }
            dys[e] = d;
        }
        __syncthreads();
        // dL/dh on the tile (dh holds gelu'(h) on entry)
        for (int e = threadIdx.x; e < HID * TILE; e += blockDim.x) {
            int c = e / TILE, j = e - c * TILE;
            float dz = 0.0f;
#pragma unroll
            for (int o = 0; o < COUT; ++o)
#pragma unroll
                for (int k = 0; k < KW; ++k)
                    dz += w[OW2 + (o * HID + c) * KW + k] * dys[o * (TILE + 4) + j + 4 - k];
            dh[e] *= dz;
        }
        __syncthreads();
        const int na = min(TILE, L - a0);
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            int p = threadIdx.x + u * NT;
            if (p >= NPAR) break;
            float s = 0.0f;
            if (p < OB1) {
                int c = p / (CIN * KW), ci = (p / KW) % CIN, k = p % KW;
                for (int j = 0; j < na; ++j) s += dh[c * TILE + j] * xs[ci * (TILE + 12) + j + k + 4];
            } else if (p < OW2) {
                int c = p - OB1;
                for (int j = 0; j < na; ++j) s += dh[c * TILE + j];
            } else if (p < OB2) {
                int q = p - OW2;
                int o = q / (HID * KW), c = (q / KW) % HID, k = q % KW;
                for (int j = 0; j < na; ++j)
                    s += dys[o * (TILE + 4) + j + 2] * zs[c * (TILE + 8) + j + k + 2];
            } else {
                int o = p - OB2;
                for (int j = 0; j < na; ++j) s += dys[o * (TILE + 4) + j + 2];
            }
            acc[u] += s;
        }
    }
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        int p = threadIdx.x + u * NT;
        if (p < NPAR) gpart[(long)t * NPAR + p] = acc[u];
    }
    __syncthreads();
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[t] = red[0];
}

// grad[p] = sum over traces in order; loss = sum of squared errors / count.
__global__ void net_reduce_kernel(const float *gpart, const float *lpart, int T, long count,
                                  float *grad, double *loss) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPAR) {
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += gpart[(long)t * NPAR + p];
        grad[p] = (float)s;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += lpart[t];
        *loss = s / (double)count;
    }
}

__global__ void net_adam_kernel(float *theta, uint16_t *pbf, float *m, float *v, const float *grad,
                                float lr, float b1, float b2, float eps, float c1, float c2) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPAR) return;
    float g = grad[p];
    float mm = b1 * m[p] + (1.0f - b1) * g;
    float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    float th = theta[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    theta[p] = th;
    pbf[p] = f32_to_bf16(th);
}

__global__ void net_set_kernel(const float *src, float *theta, uint16_t *pbf, float *m, float *v) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPAR) return;
    float th = src[p];
    theta[p] = th;
    pbf[p] = f32_to_bf16(th);
    m[p] = 0.0f;
    v[p] = 0.0f;
}

__global__ void net_get_kernel(const float *theta, const uint16_t *pbf, int rounded, float *dst) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPAR) return;
    dst[p] = rounded ? bf16_to_f32(pbf[p]) : theta[p];
}

__device__ __forceinline__ double bsum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double bmax(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// Inputs of interface i (one block each) from g_{n-1} = g1, g_{n-2} = g2 and
// the potential on the interface line (the first line of strip i+1); the
// per-trace scale s_i; and, when g0 is given, the scaled part of g0 that
// linear extrapolation misses, g0 - 2 g1 + g2.
__global__ void net_features_kernel(Phys P, const StripMeta *strips, const double2 *g1,
                                    const double2 *g2, const double2 *g0, const double *W,
                                    float *X, float *Yt, double *S) {
    __shared__ double red[256];
    const int i = blockIdx.x, ny = P.ny;
    const double2 *r1 = g1 + (long)(2 * i) * ny, *l1 = g1 + (long)(2 * i + 1) * ny;
    const double2 *r2 = g2 + (long)(2 * i) * ny, *l2 = g2 + (long)(2 * i + 1) * ny;
    const double *Wl = W + (long)strips[i + 1].line0 * ny;
    double e = 0.0, wm = 0.0;
    for (int a = threadIdx.x; a < ny; a += blockDim.x) {
        double2 r = r1[a], l = l1[a];
        e += r.x * r.x + r.y * r.y + l.x * l.x + l.y * l.y;
        wm = fmax(wm, fabs(Wl[a]));
    }
    e = bsum(e, red) / (2.0 * ny);
    wm = bmax(wm, red);
    const double s = e > 0.0 ? sqrt(e) : 1.0, is = 1.0 / s, iw = 1.0 / fmax(1.0, wm);
    if (threadIdx.x == 0) S[i] = s;
    float *x = X + (long)i * CIN * ny;
    for (int a = threadIdx.x; a < ny; a += blockDim.x) {
        double2 ra = r1[a], la = l1[a], rb = r2[a], lb = l2[a];
        x[0 * ny + a] = (float)(ra.x * is);
        x[1 * ny + a] = (float)(ra.y * is);
        x[2 * ny + a] = (float)(la.x * is);
        x[3 * ny + a] = (float)(la.y * is);
        x[4 * ny + a] = (float)(rb.x * is);
        x[5 * ny + a] = (float)(rb.y * is);
        x[6 * ny + a] = (float)(lb.x * is);
        x[7 * ny + a] = (float)(lb.y * is);
        x[8 * ny + a] = (float)(Wl[a] * iw);
        if (g0 && Yt) {
            double2 r0 = g0[(long)(2 * i) * ny + a], l0 = g0[(long)(2 * i + 1) * ny + a];
            float *y = Yt + (long)i * COUT * ny;
            y[0 * ny + a] = (float)((r0.x - 2.0 * ra.x + rb.x) * is);
            y[1 * ny + a] = (float)((r0.y - 2.0 * ra.y + rb.y) * is);
            y[2 * ny + a] = (float)((l0.x - 2.0 * la.x + lb.x) * is);
            y[3 * ny + a] = (float)((l0.y - 2.0 * la.y + lb.y) * is);
        }
    }
}

// g = 2 g1 - g2 + s * (network output), or the plain extrapolation
// 2 g1 - g2 when Y is null.
__global__ void net_guess_kernel(Phys P, const double2 *g1, const double2 *g2, const float *Y,
                                 const double *S, double2 *g) {
    const int ny = P.ny;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long n = 2L * (P.nsub - 1) * ny;
    if (e >= n) return;
    double2 b = g1[e], c = g2[e];
    double2 x = cd(2.0 * b.x - c.x, 2.0 * b.y - c.y);
    if (Y) {
        int row = (int)(e / ny), a = (int)(e - (long)row * ny);
        int i = row >> 1, side = row & 1;
        const float *y = Y + (long)i * COUT * ny;
        double s = S[i];
        x.x += s * (double)y[(2 * side) * ny + a];
        x.y += s * (double)y[(2 * side + 1) * ny + a];
    }
    g[e] = x;
}

// Per-block partials of |g - a|^2 and |g - b|^2 (two guesses judged against
// the converged vector).
__global__ void net_judge_kernel(long n, const double2 *g, const double2 *a, const double2 *b,
                                 double *part) {
    __shared__ double red[256];
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double sa = 0.0, sb = 0.0;
    if (e < n) {
        double2 x = g[e], y = a[e], z = b[e];
        sa = (x.x - y.x) * (x.x - y.x) + (x.y - y.y) * (x.y - y.y);
        sb = (x.x - z.x) * (x.x - z.x) + (x.y - z.y) * (x.y - z.y);
    }
    sa = bsum(sa, red);
    sb = bsum(sb, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa;
        part[2 * blockIdx.x + 1] = sb;
    }
}

}  // namespace

int net_nparams() { return NPAR; }

hipError_t launch_net_forward(hipStream_t st, const uint16_t *pbf, const float *X, int T, int L,
                              float *Y) {
    hipLaunchKernelGGL(net_forward_kernel, dim3((L + TILE - 1) / TILE, T), dim3(NT), 0, st, pbf, X,
                       L, Y);
    return hipGetLastError();
}

hipError_t launch_net_loss_grad(hipStream_t st, const uint16_t *pbf, const float *X,
                                const float *Yt, int T, int L, float *gpart, float *lpart,
                                float *grad, double *loss) {
    hipLaunchKernelGGL(net_train_kernel, dim3(T), dim3(NT), 0, st, pbf, X, Yt, T, L, gpart, lpart);
    hipLaunchKernelGGL(net_reduce_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, st, gpart, lpart,
                       T, (long)T * COUT * L, grad, loss);
    return hipGetLastError();
}

hipError_t launch_net_adam(hipStream_t st, float *theta, uint16_t *pbf, float *m, float *v,
                           const float *grad, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
    hipLaunchKernelGGL(net_adam_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, st, theta, pbf, m,
                       v, grad, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_net_set(hipStream_t st, const float *src, float *theta, uint16_t *pbf, float *m,
                          float *v) {
    hipLaunchKernelGGL(net_set_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, st, src, theta, pbf,
                       m, v);
    return hipGetLastError();
}

hipError_t launch_net_get(hipStream_t st, const float *theta, const uint16_t *pbf, int rounded,
                          float *dst) {
    hipLaunchKernelGGL(net_get_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, st, theta, pbf,
                       rounded, dst);
    return hipGetLastError();
}

hipError_t launch_net_features(hipStream_t st, const Phys &P, const StripMeta *strips,
                               const double2 *g1, const double2 *g2, const double2 *g0,
                               const double *W, float *X, float *Yt, double *S) {
    hipLaunchKernelGGL(net_features_kernel, dim3(P.nsub - 1), dim3(256), 0, st, P, strips, g1, g2,
                       g0, W, X, Yt, S);
    return hipGetLastError();
}

hipError_t launch_net_guess(hipStream_t st, const Phys &P, const double2 *g1, const double2 *g2,
                            const float *Y, const double *S, double2 *g) {
    long n = 2L * (P.nsub - 1) * P.ny;
    hipLaunchKernelGGL(net_guess_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, g1,
                       g2, Y, S, g);
    return hipGetLastError();
}

hipError_t launch_net_judge(hipStream_t st, long n, const double2 *g, const double2 *a,
                            const double2 *b, double *part) {
    hipLaunchKernelGGL(net_judge_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, g,
                       a, b, part);
    return hipGetLastError();
}
