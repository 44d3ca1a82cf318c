// Internal definitions of libosm: device-side metadata, launch helpers and
// the kernel launchers each translation unit provides.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Per-strip description (Section 2.1: strip j = cells [s_j, s_j + cells_j)).
struct StripMeta {
    int line0;   // global x node-line of the strip's local line 0
    int nx;      // node-lines in the strip (cells + 1)
    int off;     // first line of the strip in the packed strip layout
    int cls;     // index of its L_h block set (strips with equal nx, pl, pr share)
    double pl;   // Robin parameter on the left edge  (p, or p_bc for strip 0)
    double pr;   // Robin parameter on the right edge (p, or p_bc for strip N-1)
    // imaginary parts of the edge coefficients: the operator carries
    // i c (pl + i pl_im) M^Gamma on the left edge (likewise right); zero for
    // Robin, sum_s a_s for S_pade^m (whose real part is then pl / pr)
    double pl_im, pr_im;
};

// Mesh and equation constants passed by value to the kernels.
struct Phys {
    double hx, hy, dt, c, beta, p;
    double tre, tim;   // transmission coefficient t of S v = -i t v (+ i psi):
                       // (p, 0) for Robin, sum_s a_s for S_pade^m
    int ny;      // nodes per x-line (ncy + 1)
    int nsub;    // strips
    int nglob;   // global x node-lines (ncx + 1)
    int lt;      // packed strip lines (ncx + nsub)
};

template <typename T> struct cplx_of;
template <> struct cplx_of<double> { typedef double2 type; };
template <> struct cplx_of<float> { typedef float2 type; };

__host__ __device__ inline double2 cd(double re, double im) { double2 r; r.x = re; r.y = im; return r; }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return cd(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return cd(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return cd(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return cd(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cinv(double2 a) {
    double d = a.x * a.x + a.y * a.y;
    return cd(a.x / d, -a.y / d);
}

// Sums over the 64 lanes of a wave, the same value in every lane.  The
// lanes of each row of 16 are combined with DPP moves (VALU, no LDS
// round trip): swap neighbours, swap pairs, mirror half-rows, mirror the
// row; then the four row sums are read from lanes 0, 16, 32, 48 and added
// in that order.  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ float wave_sum_f32(float v) {
    v += __int_as_float(dpp_i32<0xB1>(__float_as_int(v)));    // quad_perm [1,0,3,2]
    v += __int_as_float(dpp_i32<0x4E>(__float_as_int(v)));    // quad_perm [2,3,0,1]
    v += __int_as_float(dpp_i32<0x141>(__float_as_int(v)));   // row_half_mirror
    v += __int_as_float(dpp_i32<0x140>(__float_as_int(v)));   // row_mirror
    const int b = __float_as_int(v);
    return (__int_as_float(__builtin_amdgcn_readlane(b, 0)) +
            __int_as_float(__builtin_amdgcn_readlane(b, 16))) +
           (__int_as_float(__builtin_amdgcn_readlane(b, 32)) +
            __int_as_float(__builtin_amdgcn_readlane(b, 48)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL>((int)b), hi = dpp_i32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Reference-element integrals of the 1-D linear shape functions psi_0 = 1-s,
// psi_1 = s on [0,1] (Section 2.2): mass, stiffness and triple product.
__device__ __forceinline__ double ref_mass(int a, int b) { return a == b ? (1.0 / 3.0) : (1.0 / 6.0); }
__device__ __forceinline__ double ref_stiff(int a, int b) { return a == b ? 1.0 : -1.0; }
__device__ __forceinline__ double ref_triple(int c, int a, int b) {
    return (a == b && b == c) ? 0.25 : (1.0 / 12.0);
}

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return the hipError_t of the launch.

struct StepCtl;   // device-side step control (kernels_control.hip); null = unguarded
struct BStrip;    // one strip of a batched solve (below)

// kernels_assemble.hip
hipError_t launch_coef(hipStream_t st, const Phys &P, const StripMeta *strips,
                       const int *line_strip, const double *W, int w_is_zero,
                       double2 *Dc, double2 *Uc, int line_begin, int line_count);
// fixed-point kernels return at once when c says the fixed point is done
// psi (may be null): per strip edge (index 2 j + side) the S_pade^m term
// sum_s a_s d_s phi_s of that edge, ny values each
hipError_t launch_residual(hipStream_t st, const Phys &P, const StripMeta *strips,
                           const int *line_strip, const double *W, const double2 *u_old,
                           const double2 *zeta, const double2 *g, double2 *res,
                           const StepCtl *c = nullptr, const double2 *psi = nullptr);
hipError_t launch_copy_u_to_strips(hipStream_t st, const Phys &P, const StripMeta *strips,
                                   const int *line_strip, const double2 *u, double2 *zeta);
hipError_t launch_update_norms(hipStream_t st, const Phys &P, double2 *zeta,
                               const double2 *delta, double *line_part,
                               const StepCtl *c = nullptr);
hipError_t launch_strip_sums(hipStream_t st, const Phys &P, const StripMeta *strips,
                             const double *line_part, double *strip_out);
// runs only once the fixed point has converged (when c is given)
hipError_t launch_flux(hipStream_t st, const Phys &P, const StripMeta *strips,
                       const double2 *g, const double2 *v, double2 *gn, double *part,
                       const StepCtl *c = nullptr, const double2 *psi = nullptr);
hipError_t launch_time_update(hipStream_t st, const Phys &P, const int2 *gline_map,
                              const double2 *v, double2 *u);
hipError_t launch_mass_partials(hipStream_t st, const Phys &P, const double2 *u, double *part);
hipError_t launch_sum(hipStream_t st, const double *part, int n, int stride, double *out);
hipError_t launch_rotating_W(hipStream_t st, const Phys &P, double xl, double yb,
                             double omega, double vxx, double vyy, double t1, double t0,
                             double *W);
hipError_t launch_check_finite(hipStream_t st, const double2 *x, long n, int *flag);
// lmax[L] = max |Re|, |Im| of b over packed line L (skipped when c says the
// fixed point is idle).  The complex-FP32 solve scales strip j by 2^-e with
// 2^e <= max over its lines < 2^(e+1), so that its right-hand side stays in
// FP32's normal range.
hipError_t launch_line_absmax(hipStream_t st, const Phys &P, const double2 *b, double *lmax,
                              const StepCtl *c);
hipError_t launch_b_line_absmax(hipStream_t st, const BStrip *strips, int nstrips, int max_nx,
                                int guard);

// kernels_factor.hip
// kind[z]: bit 0 = eliminate the line above (L-1), bit 1 = the line below (L+1)
template <typename T>
hipError_t launch_schur(hipStream_t st, int n, typename cplx_of<T>::type *F,
                        const int *lines, const int *kind, int batch,
                        const double2 *Dc, const double2 *Uc);
// In-place inversion of the Schur complements of lines[0..batch) by the
// blocked symmetric sweep, one pass (pivot block kb) per call, passes
// 0 .. sweep_passes(n)-1 in order; Pbuf: batch x 128 x 128, Rbuf/Cbuf:
// batch x 128 x n.  full != 0 leaves full storage, else upper triangles
// only.  ev0/ev1 (may be null) bracket the update kernel.
int sweep_passes(int n);
double sweep_pass_flops(int n, int kb);
template <typename T>
hipError_t launch_sweep_pass(hipStream_t st, int n, int kb, typename cplx_of<T>::type *F,
                             const int *lines, int batch, typename cplx_of<T>::type *Pbuf,
                             typename cplx_of<T>::type *Rbuf, typename cplx_of<T>::type *Cbuf,
                             int full, hipEvent_t ev0, hipEvent_t ev1);
template <typename T>
struct GemmArgs {
    int M, N, K;
    const typename cplx_of<T>::type *A; long lda; long strideA;
    const typename cplx_of<T>::type *B; long ldb; long strideB;
    const typename cplx_of<T>::type *C; long ldc;     // base (may be null or alias D)
    typename cplx_of<T>::type *D; long ldd;
    long strideCD; const int *idxCD;                   // C/D offset = (idx ? idx[z] : z) * strideCD
    int sign;                                          // D = base + sign * A * B
    int mask_lo, mask_hi;                              // base rows/cols in [lo,hi) read as zero
};
template <typename T>
hipError_t launch_zgemm(hipStream_t st, const GemmArgs<T> &g, int batch);
hipError_t launch_tridiag_apply(hipStream_t st, int n, const double2 *coef, int transpose,
                                double scale, const double2 *X, double2 *Y);
hipError_t launch_set_tridiag_mass(hipStream_t st, int n, double hy, double scale, double2 *Y);
hipError_t launch_lh_form(hipStream_t st, int n, const double2 *X, double coef_im, int add_eye,
                          double2 *out);
template <typename T>
hipError_t launch_convert(hipStream_t st, long n, const double2 *src, typename cplx_of<T>::type *dst);

// kernels_solve.hip
#define SOLVE_MAX_TEAM 64   // workgroups per strip in the solve, at most

struct SolveArgs {
    int n;
    int team;
    int shape;               // tile shape, 0 .. solve_shapes()-1 (the upper half
                             // are the kernels that read upper triangles only)
    int nstrips;
    const StripMeta *strips;
    const void *F;           // factor (double2 or float2), line stride n*n
    const double2 *Uc;       // coupling coefficients, packed lines x n x 3
    const double2 *b;        // right-hand side, packed
    double2 *x;              // solution, packed
    unsigned int *counters;  // one per strip, zero on entry
    int *error;              // set to 1 if a barrier wait times out; sticky: no
                             // solve clears it (launch_clear_flag does), and a
                             // team that finds it set stops at its next barrier
    const StepCtl *ctl;      // may be null; the whole solve is skipped when it
                             // says the fixed point is done
    int *ran;                // may be null; set to 1 when the solve was not skipped
    void *part;              // upper-triangle shapes: the members' partial buffer,
                             // nstrips x 2 x SOLVE_MAX_TEAM x 2 x n values of
                             // the factor's complex type; else unused
    const double *lmax;      // may be null (no scaling); per packed line the
                             // largest |b|: strip j's right-hand side enters the
                             // reduced-precision products as s_j b with s_j the
                             // power of two mapping its largest value into
                             // [1, 2), results leave divided by s_j
};
// ev0/ev1 (may be null) are recorded right before and after the solve kernel
hipError_t launch_strip_solve(hipStream_t st, const SolveArgs &a, int fp32, hipEvent_t ev0,
                              hipEvent_t ev1);
int solve_shapes();
int solve_max_resident_blocks(int fp32, int n, int shape);
// 1 for the shapes of the upper-triangle (half-storage) solve kernels
int solve_shape_is_sym(int shape);
// 1 when the half-storage solve has a kernel for n and fits the device's LDS
int solve_sym_supported(int n, int fp32);
size_t solve_pf_smem(int n, int fp32);

// kernels_yorder.hip: the strip factor and solve in y-line order (the
// strip's unknowns taken y-line by y-line: blocks of its nx node-lines,
// block tridiagonal along the ny y-lines), twisted, formed in FP64; the
// inverses stored in FP64 or (fp32) complex FP32; Robin only.
#define YORDER_MAX_NX 64
struct YStrip {
    int off;     // first packed line of the strip
    int nx;      // node-lines of the strip (<= YORDER_MAX_NX)
    long yoff;   // first element of its inverses in the factor: ny x nx x nx
    long boff;   // first element of its coupling coefficients: (ny - 1) x 3 x nx
                 // (per y-line a: B_a's diagonal, upper and lower entries)
};
size_t yorder_factor_lds(int max_nx);
// algorithmic flops of factoring one strip (ny y-lines of nx unknowns)
double yorder_factor_flops(int ny, int nx);
// Dc, Uc: coefficients of every packed line (launch_coef layout); writes the
// inverses (YF: double2, or float2 when fp32) and the coupling coefficients
// in y-line order (YB)
hipError_t launch_yfactor(hipStream_t st, const YStrip *ys, int nstrips, int ny, int max_nx,
                          const double2 *Dc, const double2 *Uc, void *YF, int fp32, double2 *YB,
                          hipEvent_t ev0, hipEvent_t ev1);
// x = K^{-1} b on every strip; skipped when c says the fixed point is done
// (ran, when given, set to 1 otherwise); ev0/ev1 bracket the three kernels.
// prog: 2 nstrips progress words (zeroed once; the sweeps' L2 prefetch
// helpers poll them), epoch: the host's launch counter for them (advanced
// by two per call, below 2^44)
hipError_t launch_ysolve(hipStream_t st, const YStrip *ys, int nstrips, int ny, int max_nx,
                         const void *YF, int fp32, const double2 *YB, const double2 *b,
                         double2 *x, const StepCtl *c, int *ran, unsigned long long *prog,
                         unsigned long long *epoch, hipEvent_t ev0, hipEvent_t ev1);

// kernels_control.hip
// Step configuration and device-side state of one time step.
struct StepCfg {
    double tol_q, eta_q, tol_k;
    int tol_k_rel, fixed_q, max_q, fixed_k, classical;
    int q_est;      // error-estimate fixed-point test (osm_options.q_estimate)
};
struct StepCtl {
    StepCfg cfg;
    int q_conv;     // fixed point of the current Schwarz map converged
    int q_iter;     // fixed-point iterations of the current Schwarz map
    int q_total;    // summed over the step
    int q_fail;     // max_q reached without convergence
    int r_done;     // 1: Schwarz map evaluated, 2: preconditioned update done
    int k;          // Schwarz iterations completed
    int k_done;     // Schwarz iteration converged
    int bad;        // non-finite value met
    int commit;     // classical: g <- R(g) pending
    int gm_total;   // GMRES iterations summed over the step
    int ready;      // a new Schwarz iteration may start (batched replay)
    double tq;      // fixed-point tolerance of the current Schwarz map
    double inc, ref, prev_rel;
    double first_rel;  // relative increment of the first Schwarz iteration of the
                       // last step (kept across steps; 0 = none yet)
    double rho;        // largest contraction ratio measured in this step (0 = none)
};
struct GmresCtl;
// g[k] = u(2k) + i u(2k+1), u(j) uniform on [0, 1) from the (j+1)-th output of
// SplitMix64 seeded with `seed` (Section 5: a random first interface vector)
hipError_t launch_random_interface(hipStream_t st, double2 *g, long n, uint64_t seed);
hipError_t launch_step_init(hipStream_t st, StepCtl *c, const StepCfg &cfg);
hipError_t launch_iter_reset(hipStream_t st, StepCtl *c, GmresCtl *g);
hipError_t launch_copy_u_guarded(hipStream_t st, const Phys &P, const StripMeta *strips,
                                 const int *line_strip, const double2 *u, double2 *zeta,
                                 const StepCtl *c);
// dprev (may be null): per-strip ||zeta^q - zeta^{q-1}||^2 of the previous
// iterate, kept for the contraction estimate of the error-estimate test
hipError_t launch_q_check(hipStream_t st, const Phys &P, const StripMeta *strips,
                          const double *part, StepCtl *c, double *dprev = nullptr);
hipError_t launch_flux_finalize(hipStream_t st, const double *part, int nt, StepCtl *c);
hipError_t launch_commit(hipStream_t st, long n, double2 *g, const double2 *gn, const StepCtl *c);
hipError_t launch_precond_rhs(hipStream_t st, long n, const double2 *g, const double2 *gn,
                              double2 *y, double2 *x, const StepCtl *c);
hipError_t launch_precond_update(hipStream_t st, long n, double2 *g, const double2 *x,
                                 double *part, const StepCtl *c, const GmresCtl *gc);

// kernels_gmres.hip
// Device-side state of one GMRES solve (Arnoldi loop driven on the GPU).
struct GmresCtl {
    int done;       // cycle finished: converged, breakdown or non-finite
    int conv;       // residual estimate met tol * bnorm
    int bad;        // non-finite value met
    int j;          // Arnoldi steps completed in this cycle
    int finished;   // x updated from this cycle
    int total;      // Arnoldi steps summed over the cycles of this solve
    int skip;       // the current end-of-cycle launch does nothing
    double bnorm;   // ||y||
    double tol;     // relative tolerance
    double beta;    // ||r_0|| of the cycle
    double inv_hn;  // 1 / h_{j+1,j} (normalisation of the next basis vector)
    double resid;   // current residual estimate
};
// Host-visible copy of the step's control state: one small kernel writes
// the step control, the GMRES control (when g is given) and the solve's error
// flag into pinned host memory, so the host reads all three after one
// synchronisation instead of three device-to-host copies.
struct CtlMirror {
    StepCtl s;
    GmresCtl g;
    int err;
    int flag;     // launch_scalar_gather: a device flag
    double val;   // launch_scalar_gather: a device scalar
};
hipError_t launch_ctl_gather(hipStream_t st, const StepCtl *s, const GmresCtl *g, const int *err,
                             CtlMirror *out);
// copies *flag (when given) and *val into out->flag and out->val
hipError_t launch_scalar_gather(hipStream_t st, const int *flag, const double *val,
                                CtlMirror *out);
// sctl (may be null): the cycle starts only when the Schwarz map of the
// current iteration has been evaluated.
hipError_t launch_gmres_begin(hipStream_t st, long n, const double2 *r, double *norm_part,
                              int first, double accept, double2 *V0, double2 *e, int m,
                              GmresCtl *ctl, const StepCtl *sctl);
// chunks of the Gram-Schmidt partial dot products for vectors of length n
// (part buffers hold gmres_chunks(n) x (m + 1) values)
int gmres_chunks(long n);
// Work plan of the register-resident L_h kernel (built once per handle).
// Class c of the plan (classes ordered by decreasing strips per workgroup,
// so the longest workgroups are dispatched first) owns the workgroups
// [block_off, block_off + tiles * groups): `groups` strip groups for every
// row tile.  Its `count` strips are list[list_off ...] in increasing index,
// and group g takes the ranks g, g + groups, ...
struct LhClass {
    int cls, list_off, count, groups, block_off;
};
// L_h in the eigenbasis of the y-direction (kernels_lhmodal.hip): used
// instead of the dense blocks when phi is set.
struct LhModal {
    const double *phi = nullptr;     // n x n, Phi[j][mu]
    const double *phinv = nullptr;   // n x n, Phi^{-1}[mu][j]
    const double2 *dm = nullptr;     // ncls x 4 x n: the modal diagonals of X^1 .. X^4
    double2 *xh = nullptr;           // 2 x 2 (N - 1) x n work vectors (transformed traces,
                                     // then their per-mode combination)
    int lg = 0;                      // > 0: the transforms by FFT of length 2^lg = 2 (n - 1)
};
struct LhPlan {
    const LhClass *tab = nullptr;   // device, ncls entries
    const int *list = nullptr;      // device, nsub entries
    int ncls = 0, tiles = 0;
    int blocks = 0;                 // 0: the register-resident kernel is not used
    LhModal md;
};
// kernels_lhmodal.hip: y = L_h x, or x - L_h x when mode_p (x, y distinct,
// interface layout); skipped when ctl says the GMRES cycle is done
hipError_t launch_lh_modal(hipStream_t st, const Phys &P, const StripMeta *strips,
                           const LhModal &md, const double2 *x, double2 *y, int mode_p,
                           const GmresCtl *ctl);
// log2 of the FFT length 2 (n - 1) when n - 1 is a power of two in [4, 2048],
// else 0; the dynamic LDS of the FFT kernels at that length
int lh_fft_log2(int n);
size_t lh_fft_lds(int lg);
// the dense n x n block X^{blk} of strip class cls from the modal form
hipError_t launch_lh_modal_dense(hipStream_t st, int n, const LhModal &md, int cls, int blk,
                                 double2 *out);
// Host side of the plan: strip_cls[j] is strip j's class.  Fills tab and
// list and returns the workgroup count (0 when ny needs more than 17 column
// chunks).
int lh_plan_build(int ny, int nsub, const int *strip_cls, int ncls, std::vector<LhClass> &tab,
                  std::vector<int> &list);
// an upper bound of lh_plan_build's workgroup count from the sizes alone
int lh_fused_blocks_bound(int ny, int nsub, int ncls);
// One Arnoldi step j.  mvpart (may be null): pl.blocks x (m + 1) partials of
// the fused three-kernel form, used when pl.blocks > 0 and j < 64;
// otherwise the six-kernel form (matvec, dots, two updates, rotation,
// normalisation).
hipError_t launch_gmres_iteration(hipStream_t st, const Phys &P, const StripMeta *strips,
                                  int ncls, const LhPlan &pl, const double2 *LH, long n, int j,
                                  int m, double2 *V, double2 *part1, double2 *part2,
                                  double *norm_part, double2 *H, double2 *cs, double2 *sn,
                                  double2 *e, GmresCtl *ctl, double2 *mvpart);
hipError_t launch_gmres_finish(hipStream_t st, long n, int m, const double2 *H, const double2 *e,
                               double2 *y, const double2 *V, double2 *x, GmresCtl *ctl,
                               int require_done);
hipError_t launch_lh_matvec(hipStream_t st, const Phys &P, const StripMeta *strips, int ncls,
                            const LhPlan &pl, const double2 *LH, const double2 *x, double2 *y,
                            int mode_p);
hipError_t launch_multidot(hipStream_t st, long n, const double2 *V, int nv, const double2 *w,
                           double2 *part, int nblk);
hipError_t launch_multidot_finalize(hipStream_t st, const double2 *part, int nv, int nblk,
                                    double2 *out);
hipError_t launch_multiaxpy(hipStream_t st, long n, const double2 *V, int nv, const double2 *h,
                            double2 *w, int sub);
hipError_t launch_norm_partials(hipStream_t st, long n, const double2 *x, double *part, int nblk);
hipError_t launch_scale_copy(hipStream_t st, long n, const double2 *x, double2 s, double2 *y);
hipError_t launch_axpby(hipStream_t st, long n, double2 a, const double2 *x, double2 b,
                        const double2 *y, double2 *z);

// kernels_pade.hip: the S_pade^m condition on the 2 nsub strip edges (edge
// 2 j + side, side 0 = the strip's first line); ad = (a_s, d_s) pairs; sub,
// cp, inv: LU of each D_{e,s} (edge-major, ny values per (e, s)); the free
// edge (W = 0, for L_h) has index nedge.
// (edges e_first .. nedge - 1, and the free edge when with_free)
hipError_t launch_pade_lu(hipStream_t st, const Phys &P, const StripMeta *strips, const double *W,
                          int nedge, int with_free, int m, const double2 *ad, double2 *sub,
                          double2 *cp, double2 *inv, int e_first = 0);
// G_e = scale sum_s a_s d_s D_{e,s}^{-1} M^G for edges [e0, e0 + ecount),
// into G (ecount x ny x ny); X: ecount x ny x ny scratch
hipError_t launch_pade_G(hipStream_t st, int ny, double hy, int e0, int ecount, int m,
                         const double2 *ad, const double2 *sub, const double2 *cp,
                         const double2 *inv, double2 *X, double2 *G, double2 scale);
// F[lines[b]] += -i c M^G G_{edges[b]} on the upper tiles, b < batch
template <typename T>
hipError_t launch_pade_edge_add(hipStream_t st, int n, typename cplx_of<T>::type *F,
                                const int *lines, const int *edges, int batch, int e0,
                                const double2 *G, double c, double hy);
// fixed point: z and the eliminated edge right-hand side added to res ...
hipError_t launch_pade_fp_residual(hipStream_t st, const Phys &P, const StripMeta *strips,
                                   const double *W, int nedge, int m, const double2 *ad,
                                   const double2 *sub, const double2 *cp, const double2 *inv,
                                   const double2 *zeta, const double2 *phi, double2 *z,
                                   double2 *res, const StepCtl *c);
// ... and, after the strip solve (delta), the edge functions and psi
hipError_t launch_pade_fp_update(hipStream_t st, const Phys &P, const StripMeta *strips, int nedge,
                                 int m, const double2 *ad, const double2 *sub, const double2 *cp,
                                 const double2 *inv, const double2 *delta, const double2 *z,
                                 double2 *phi, double2 *work, double2 *psi, const StepCtl *c);
hipError_t launch_pade_reset(hipStream_t st, long nphi, double2 *phi, long npsi, double2 *psi,
                             const StepCtl *c);
// out = -2i sa X (- I when add_eye)
hipError_t launch_pade_lh_form(hipStream_t st, int n, const double2 *X, double2 sa, int add_eye,
                               double2 *out);

// kernels_krylov.hip: BiCGStab for P x = y (P = I - L_h) with device-side
// scalars; ctl carries done / conv / finished / bad / total as for GMRES.
// V holds the 6 work vectors r, rh, p, v, s, t (6 n values); part holds
// bicg_partials() doubles.
struct BicgState {
    double2 rho, alpha, omega, beta;
};
int bicg_partials();
hipError_t launch_bicg_start(hipStream_t st, long n, const double2 *y, double2 *x, double2 *V,
                             double *part, BicgState *S, GmresCtl *ctl, const StepCtl *sc);
hipError_t launch_bicg_iteration(hipStream_t st, const Phys &P, const StripMeta *strips, int ncls,
                                 const LhPlan &pl, const double2 *LH, long n, double2 *V,
                                 double2 *x, double *part, BicgState *S, GmresCtl *ctl,
                                 const StepCtl *sc, int max_it);

// ---------------------------------------------------------------- batched instances
// One entry per independent instance of a batch: its mesh constants and the
// device buffers of its strips, interfaces and step control.  Batched kernels
// take instance blockIdx.z (or blockIdx.y / blockIdx.x for per-line /
// per-instance kernels) from this table; the grids cover the largest
// instance and smaller instances return early.
struct InstDesc {
    Phys P;
    const StripMeta *strips;
    const int *line_strip;
    const int2 *gmap;
    const double *W;
    double2 *u;                     // u_{n-1} in, u_n out (global nodes)
    double2 *zeta, *res, *delta;    // packed strip vectors
    double2 *g, *gn;                // interface vectors
    double *line_part, *trace_part, *mass_part;
    double *scal;                   // [0] mass before, [1] mass after
    StepCtl *ctl;
    GmresCtl *gctl;                 // preconditioned instances: reset with the iteration
    int *flag;                      // non-finite input
};

// One strip of a batched solve: pointers already offset to the strip's
// first packed line.
struct BStrip {
    const void *F;          // stored inverses (double2 or float2), n*n per line
    const double2 *Uc;      // coupling coefficients, n*3 per line
    const double2 *b;       // right-hand side
    double2 *x;             // solution
    const StepCtl *ctl;     // the instance's control; solve skipped when idle
    double *lmax;           // may be null (no scaling); largest |b| of each of
                            // the strip's lines (scale as in SolveArgs::lmax)
    int n, nx;
};
// One work item: member `member` of the `team` workgroups solving `strip`.
// The members of a strip are consecutive items.
struct BItem {
    int strip, member, team, pad;
};
struct BatchSolveArgs {
    const BStrip *strips;
    const BItem *items;
    const int *nitems;      // device: the live item count (the host may re-plan
                            // the items between launches)
    int nstrips;
    unsigned *counters;     // nstrips barrier counters, then the queue head
    int *error;             // sticky, as SolveArgs::error
    int *ran;               // may be null; set to 1 when any strip was solved
    unsigned long long *work;  // may be null; algorithmic bytes of the strips solved
    int guard;              // 1: skip strips whose instance's fixed point is idle
};
struct BatchDims {
    int nb, max_ny, max_lt, max_nglob, max_ntr;
    long max_ng;
};
// kernels_batch.hip
hipError_t launch_b_check_finite(hipStream_t st, const InstDesc *tab, const BatchDims &d);
hipError_t launch_b_mass(hipStream_t st, const InstDesc *tab, const BatchDims &d, int slot);
hipError_t launch_b_step_init(hipStream_t st, const InstDesc *tab, const BatchDims &d,
                              const StepCfg &cfg);
hipError_t launch_b_copy_u(hipStream_t st, const InstDesc *tab, const BatchDims &d, int guarded);
hipError_t launch_b_iter_reset(hipStream_t st, const InstDesc *tab, const BatchDims &d);
hipError_t launch_b_residual(hipStream_t st, const InstDesc *tab, const BatchDims &d);
hipError_t launch_b_update_norms(hipStream_t st, const InstDesc *tab, const BatchDims &d);
hipError_t launch_b_q_check(hipStream_t st, const InstDesc *tab, const BatchDims &d);
hipError_t launch_b_flux(hipStream_t st, const InstDesc *tab, const BatchDims &d);
hipError_t launch_b_commit(hipStream_t st, const InstDesc *tab, const BatchDims &d);
hipError_t launch_b_time_update(hipStream_t st, const InstDesc *tab, const BatchDims &d);
// kernels_solve.hip: variant = tile shape index (0 .. batch_solve_variants()-1)
// *flag = 0 on the stream (a kernel, so the call may sit in a captured graph)
hipError_t launch_clear_flag(hipStream_t st, int *flag);
hipError_t launch_batch_solve(hipStream_t st, const BatchSolveArgs &a, int fp32, int variant,
                              int grid, int max_n, hipEvent_t ev0, hipEvent_t ev1);
int batch_solve_variants();
const char *batch_solve_variant_name(int fp32, int variant);
int batch_solve_max_resident_blocks(int fp32, int variant, int max_n);

// ---------------------------------------------------------------- learned guess
// kernels_net.hip: network conv1d(9->64,k5) -> GELU -> conv1d(64->4,k5) over
// interface lines; bf16 parameter copy, FP32 master, FP32 accumulation.
int net_nparams();
hipError_t launch_net_forward(hipStream_t st, const uint16_t *pbf, const float *X, int T, int L,
                              float *Y);
hipError_t launch_net_loss_grad(hipStream_t st, const uint16_t *pbf, const float *X,
                                const float *Yt, int T, int L, float *gpart, float *lpart,
                                float *grad, double *loss);
hipError_t launch_net_adam(hipStream_t st, float *theta, uint16_t *pbf, float *m, float *v,
                           const float *grad, float lr, float b1, float b2, float eps, float c1,
                           float c2);
hipError_t launch_net_set(hipStream_t st, const float *src, float *theta, uint16_t *pbf, float *m,
                          float *v);
hipError_t launch_net_get(hipStream_t st, const float *theta, const uint16_t *pbf, int rounded,
                          float *dst);
// inputs (nsub-1, 9, ny), scales (nsub-1) and, when g0 and Yt are given, the
// targets (nsub-1, 4, ny)
hipError_t launch_net_features(hipStream_t st, const Phys &P, const StripMeta *strips,
                               const double2 *g1, const double2 *g2, const double2 *g0,
                               const double *W, float *X, float *Yt, double *S);
// g = 2 g1 - g2 + S * Y (network output), or the linear extrapolation 2 g1 - g2 when Y is null
hipError_t launch_net_guess(hipStream_t st, const Phys &P, const double2 *g1, const double2 *g2,
                            const float *Y, const double *S, double2 *g);
hipError_t launch_net_judge(hipStream_t st, long n, const double2 *g, const double2 *a,
                            const double2 *b, double *part);
