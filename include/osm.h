/*
 * osm.h -- C ABI of the MI355X optimized-Schwarz solver for the 2-D nonlinear
 * Schroedinger / Gross-Pitaevskii equation (Besse & Xing, arXiv:1603.05110).
 *
 * One call of osm_step advances the Duran-Sanz-Serna midpoint scheme by one
 * time step (Section 2.1, eq. CNS): the stationary nonlinear problem of the
 * step is split into non-overlapping x-strips (Section 2.1, eq. algolocal)
 * coupled by Robin transmission conditions S = -ip (eq. TCSRobin), each strip
 * problem is resolved by the fixed point of Section 2.2 (eq. localpbrobin) on
 * the Q1 finite-element system of eq. NproblemRobinNL, and the interface
 * vector g = (r_1, l_2, r_2, ..., l_N) (eq. algo_d) is iterated either by the
 * classical algorithm g <- R(g) (eqs. fluxlr, AlgoGraph) or by the
 * preconditioned algorithm g <- g - P^{-1}(g - R(g)) with P = I - L_h
 * (Section 3, eqs. algo_pd, Lmpi), P^{-1} applied by GMRES (Section 4.2).
 *
 * Conventions shared by every entry point
 *   - Mesh: ncx x ncy cells on (xl,xr) x (yb,yu); nodal arrays are x-major,
 *     y-fast, (ncx+1)*(ncy+1) entries, node (i,k) at (xl+i*hx, yb+k*hy).
 *   - Strip j owns cells [s_j, s_j + strip_cells[j]) in x and the node-lines
 *     s_j .. s_j+strip_cells[j]; interface lines are duplicated.  "Packed
 *     strip layout" = the strips' node-lines concatenated in strip order,
 *     (ncx + nsub) lines of ny = ncy+1 complex values.
 *   - Interface vectors have shape (2*(nsub-1), ny): row 2i is r_i, row 2i+1
 *     is l_{i+1}, for the interface between strips i and i+1 (0-based).
 *   - Complex values are osm_c64 = {re, im} (the layout of torch.complex128).
 *   - Pointers named *_dev are device pointers on the handle's device, valid
 *     and 16-byte aligned for the duration of the call; the caller owns them.
 *     Host structs are read during the call and copied where needed.
 *   - All work is enqueued on the HIP stream given to osm_setup; entry points
 *     that report scalars (stats, norms) synchronise that stream.
 *   - Every call returns an osm_status; nothing throws or aborts across the
 *     ABI.  On error the message is available from osm_last_error.
 *     OSM_EINVAL leaves outputs untouched; OSM_ENOCONV leaves u_dev holding
 *     u_{n-1} unchanged and fills the stats.
 */
#ifndef OSM_H
#define OSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct osm_handle osm_handle;
typedef struct osm_net osm_net;
typedef struct { double re, im; } osm_c64;

typedef enum {
    OSM_OK = 0,
    OSM_EINVAL = -1,        /* bad argument (sizes, strips, parameters)         */
    OSM_ENOMEM = -2,        /* footprint exceeds free device memory or the cap  */
    OSM_EHIP = -3,          /* a HIP runtime call or kernel launch failed       */
    OSM_ENOCONV = -4,       /* fixed point, Schwarz or GMRES hit its cap        */
    OSM_ENONFINITE = -5,    /* NaN/Inf met in the iterates                      */
    OSM_ESTATE = -6,        /* call out of order (e.g. step before factor)      */
    OSM_EUNSUPPORTED = -7   /* option not built (e.g. the Pade condition)       */
} osm_status;

typedef enum { OSM_TC_ROBIN = 0, OSM_TC_PADE = 1 } osm_tc;
typedef enum {
    OSM_CLASSICAL = 0,          /* g <- R(g) (eqs. fluxlr, AlgoGraph)              */
    OSM_PRECOND = 1,            /* g <- g - P^{-1}(g - R(g)) (eq. algo_pd)         */
    OSM_INTERFACE_KRYLOV = 2    /* f = 0 only: R is affine, R(g) = L g + d, and the
                                   interface problem (I - L) g = d (eq.
                                   interfacepb_d) is solved by restarted GMRES
                                   whose every product is one Schwarz map (all
                                   strip solves); stats.k counts Schwarz maps,
                                   stats.gmres_total GMRES iterations; stopping
                                   rule ||residual|| < tol_k (x ||d|| when
                                   tol_k_relative)                              */
} osm_algo;
typedef enum { OSM_FP64 = 0, OSM_C32_REFINE = 1 } osm_prec;
typedef enum {
    OSM_IFACE_R = 0,          /* g_out = R(g_in): the nonlinear Schwarz map      */
    OSM_IFACE_I_MINUS_R = 1,  /* g_out = g_in - R(g_in)                          */
    OSM_IFACE_LH = 2,         /* g_out = L_h g_in (free linear part, eq. Lmpi)  */
    OSM_IFACE_PINV = 3        /* g_out = (I - L_h)^{-1} g_in by GMRES            */
} osm_iface_op;

/* The problem statement (Section 2: eqs. Sch, BC, BCRobin; Section 2.1). */
typedef struct {
    double xl, xr, yb, yu;        /* Omega = (xl,xr) x (yb,yu)                    */
    int32_t ncx, ncy;             /* cells per direction                          */
    int32_t nsub;                 /* N x-strips (>= 2)                            */
    const int32_t *strip_cells;   /* host, nsub entries >= 2 summing to ncx;
                                     NULL = equal strips (ncx % nsub == 0)        */
    double lap_coef;              /* c in i u_t + c Lap u + V u + f(u) u = 0:
                                     1 (NLS) or 1/2 (GPE, Section 5.2)            */
    double beta;                  /* f(u) = beta |u|^2, sign as in eq. Sch        */
    int32_t tc;                   /* osm_tc: OSM_TC_ROBIN, or OSM_TC_PADE for the
                                     absorbing condition S_pade^m of eq. TCS (with
                                     eq. TCS_phi) on every interface and on the
                                     physical x-edges (eq. BC with eq. BCS2p);
                                     p and p_bc are then not used                 */
    double p;                     /* Robin transmission parameter, S = -ip, p > 0  */
    double p_bc;                  /* Robin parameter on the physical x-edges
                                     (the paper uses p_bc = p; 0 = Neumann)        */
    double dt;                    /* time step                                     */
    double omega, vxx, vyy;       /* rotating-frame potential (Section 5.2.1):
                                     V(x,y) = vxx x^2 + vyy y^2 seen at A(t) x~;
                                     used only by osm_factor_rotating              */
    int32_t pade_m;               /* OSM_TC_PADE: number of terms m (1 .. 512) of
                                     a_s = e^{i theta/2} / (m cos^2((2s-1)pi/(4m))),
                                     d_s = e^{i theta} tan^2((2s-1)pi/(4m)),
                                     s = 1 .. m (the sums of eq. TCS start at 1)   */
    double pade_theta;            /* branch-cut rotation theta in (0, pi); the
                                     paper takes pi/4                              */
} osm_problem;

typedef struct {
    int32_t algo;                 /* osm_algo                                      */
    int32_t prec;                 /* osm_prec: FP64, or complex-FP32 factor and
                                     substitution with FP64 residual correction    */
    double tol_k;                 /* Schwarz stop: ||g^{k+1}-g^k||_2 < tol_k
                                     (paper: 1e-10 absolute, Section 5)            */
    int32_t tol_k_relative;       /* 1: tol_k * ||g^{k+1}||_2 instead             */
    int32_t max_k;
    double tol_q;                 /* fixed point: ||dzeta|| <= tol_q ||zeta||.  The
                                     fixed point of eq. localpbrobin is run in
                                     residual form, zeta <- zeta + K(W)^{-1} (F -
                                     K(W + beta|zeta|^2) zeta), with K(W) factored
                                     once per W_n: with an exact K(W)^{-1} this is
                                     the nonlinearity-on-the-right form the paper
                                     writes for S_pade (eq. NproblemSPNL), and it
                                     has the fixed point of eq. NproblemRobinNL.
                                     The form is fixed; there is no switch.      */
    int32_t max_q;
    int32_t fixed_k, fixed_q;     /* > 0: run exactly that many iterations         */
    int32_t warm_start;           /* 1: each fixed point starts from the previous
                                     Schwarz iterate; 0: from u_{n-1} (paper)      */
    double tol_gmres;             /* relative residual of P x = y                  */
    int32_t gmres_restart, max_gmres;
    int32_t guess;                /* 0: g_n^0 = g_{n-1} converged (paper);
                                     1: the vector of osm_set_interface_guess;
                                     2: learned prediction (osm_set_guess_net);
                                     3: linear extrapolation 2 g_{n-1} - g_{n-2}.
                                     2 and 3 start once two converged vectors
                                     exist; a prediction that ended farther from
                                     g_n than g_{n-1} did disables the next one,
                                     and a step that fails from a prediction is
                                     restarted from g_{n-1}, and the step after it
                                     starts from its g_{n-1} (stats.fallback_used) */
    int32_t team;                 /* workgroups per strip in the solve; 0 = auto   */
    uint64_t mem_cap;             /* 0 = free device memory; else a byte cap       */
    double eta_q;                 /* > 0: inexact inner solves; Schwarz iteration k
                                     stops its fixed points at
                                     max(tol_q, eta_q * (relative increment of
                                     iteration k-1)), iteration 1 at
                                     max(tol_q, eta_q); the converged answer is
                                     unchanged.  0 = always tol_q                 */
    int32_t solve_shape;          /* 0 = the autotuner picks the strip solve's kernel
                                     and tile shape; k = 1 .. 8 fixes shape k-1:
                                     0 .. 3 read full rows of the stored inverses,
                                     4 .. 7 only their upper triangles (the
                                     inverses are complex symmetric; ny up to 2112
                                     in c32, 1088 in FP64); the team is still tuned
                                     unless team > 0                             */
    int32_t q_estimate;           /* 0: a fixed point stops when ||zeta^q - zeta^{q-1}||
                                     <= tol ||zeta^q|| on every strip (the paper's
                                     test).  1: from the second Schwarz iteration
                                     of a step on, it also stops when the error
                                     bound r/(1-r) ||zeta^q - zeta^{q-1}|| of a
                                     contraction is below tol ||zeta^q||, with r
                                     twice the largest ratio ||zeta^2 - zeta^1|| /
                                     ||zeta^1 - zeta^0|| over the strips measured
                                     in the step (used only while r < 1/2); the
                                     converged answer is unchanged              */
    int32_t g1_init;              /* first step's interface start g_1^0 (Section 5,
                                     initial vectors): 0 = zero; 1 = seeded random,
                                     entry k of the interface array (row-major) is
                                     u(2k) + i u(2k+1) with u(j) uniform on [0, 1)
                                     from the (j+1)-th output of SplitMix64
                                     seeded with `seed` (the top 53 bits times
                                     2^-53).  Instance b of a batch uses seed + b. */
    uint64_t seed;
    int32_t krylov;               /* solver of P x = y in OSM_PRECOND (Section 4.2
                                     names GMRES or BiCGStab): 0 = restarted
                                     GMRES, 1 = BiCGStab (needs gmres_restart >= 4,
                                     its work vectors share the GMRES basis);
                                     stats.gmres_total then counts BiCGStab
                                     iterations                                   */
    int32_t strip_order;          /* unknown order of the strip factor (Section 2.2:
                                     K_j is block tridiagonal in either order):
                                     0 = node-line order, ny x ny blocks, dense
                                     Schur complements inverted on the matrix
                                     cores (as in prec); 1 = y-line order, nx x nx
                                     blocks (nx = a strip's node-lines) along the
                                     ny y-lines, complements formed and inverted
                                     in FP64, the inverses stored as prec says
                                     (complex FP32 in OSM_C32_REFINE) and applied
                                     in FP64 (Robin only, every strip at most 64
                                     node-lines; EINVAL otherwise);
                                     2 = the autotuner times one solve of each
                                     order after the first factorisation and
                                     keeps the faster (node-line order where the
                                     y-line order is not available; both factors
                                     are allocated).  osm_strip_order() tells
                                     which is in use.                             */
    int32_t lh_form;              /* OSM_PRECOND, how L_h is kept and applied:
                                     1 = dense ny x ny blocks per strip class,
                                     built at setup by 2 ny strip solves each
                                     (the form S_pade^m always uses); 2 = for
                                     the Robin condition, in the cosine
                                     eigenbasis of the y-direction (exact for
                                     W = 0 on the uniform mesh: a discrete
                                     cosine transform of every trace, a 2 x 2
                                     combination per mode, the transform back;
                                     by FFT of length 2 (ny - 1) when ny - 1 is
                                     a power of two up to 2048, else as dense
                                     real ny x ny products on the matrix
                                     cores); 0 = 2 where ny - 1 is such a power
                                     of two at least 1024 or where the dense
                                     blocks' fused product kernel does not
                                     apply (ny > 1088), else 1                   */
} osm_options;

typedef struct {
    int32_t k;                    /* Schwarz (outer) iterations                    */
    int32_t q_total;              /* fixed-point iterations summed over k          */
    int32_t gmres_total;          /* GMRES iterations summed over k                */
    int32_t refine_total;         /* FP32 solves corrected by an FP64 residual     */
    int32_t fallback_used;        /* 0: the start mode's vector was used; 1: the
                                     prediction was rejected before the step (the
                                     last judge found it worse than g_{n-1}), g_{n-1}
                                     used; 2: the step failed from the prediction and
                                     was restarted from g_{n-1}                     */
    double last_increment;        /* last ||g^{k+1} - g^k||_2                      */
    double mass_before, mass_after; /* u* M u before and after the step           */
    double guess_ratio;           /* guess 2 or 3, once a prediction was formed:
                                     ||g_n - prediction|| / ||g_n - g_{n-1}|| (the
                                     fallback's judge; < 1: the prediction was the
                                     closer start), g_n the converged vector; 0
                                     otherwise                                    */
} osm_step_stats;

typedef struct { uint64_t device_bytes, host_bytes; } osm_footprint;

/* Device and host bytes osm_setup would allocate.  Pure host computation. */
osm_status osm_query(const osm_problem *prob, const osm_options *opt,
                     osm_footprint *out);

/* Validate the problem, allocate every device buffer (the only allocation
 * point), build the free interface operator L_h when opt->algo is
 * OSM_PRECOND (Section 4.2: 2 ny single-strip solves per distinct strip),
 * and return a handle bound to hip_stream (NULL = default stream) and to the
 * current device.  Returns OSM_ENOMEM before allocating when the footprint
 * exceeds the free device memory or opt->mem_cap. */
osm_status osm_setup(const osm_problem *prob, const osm_options *opt,
                     void *hip_stream, osm_handle **out);

/* Set the step potential W_n = (V_n + V_{n-1})/2 (Section 2.1) from a device
 * array of (ncx+1)*(ncy+1) doubles and factor every strip operator
 * K_j(W_n) = 2i/dt M - c S + M_W + i c (p_l M^Gamma_l + p_r M^Gamma_r)
 * (eq. NproblemRobinNL without the nonlinear term) by block Thomas with dense
 * ny x ny Schur complements, inverted on the matrix cores. */
osm_status osm_factor(osm_handle *h, const double *W_dev);

/* Same, with W_n computed on the device from the rotating-frame potential of
 * Section 5.2.1 at t_n = n dt and t_{n-1}. */
osm_status osm_factor_rotating(osm_handle *h, int32_t n);

/* One time step: u_dev holds u_{n-1} (global nodes) on entry and u_n on
 * successful exit.  stats may be NULL. */
osm_status osm_step(osm_handle *h, osm_c64 *u_dev, osm_step_stats *stats);

/* Interface operators at the state u_dev = u_{n-1} (read only; ignored for
 * OSM_IFACE_LH and OSM_IFACE_PINV).  g_in_dev and g_out_dev have the
 * interface layout and must not overlap. */
osm_status osm_interface_apply(osm_handle *h, osm_iface_op op,
                               const osm_c64 *u_dev, const osm_c64 *g_in_dev,
                               osm_c64 *g_out_dev);

/* Interface guess g^0 for the next osm_step when opt->guess == 1. */
osm_status osm_set_interface_guess(osm_handle *h, const osm_c64 *g0_dev);

/* Copy the last converged interface vector. */
osm_status osm_get_interface(osm_handle *h, osm_c64 *g_dev);

/* x = K_j(W_n)^{-1} b on every strip at once (packed strip layout), with the
 * factor of the last osm_factor in the handle's precision (FP32 factors are
 * applied without correction).  b_dev and x_dev must not overlap. */
osm_status osm_strip_solve(osm_handle *h, const osm_c64 *b_dev, osm_c64 *x_dev);

/* Copy the strip solutions v_j of the last step or interface apply (packed
 * strip layout). */
osm_status osm_get_strip_solution(osm_handle *h, osm_c64 *v_dev);

/* Copy the dense blocks X^{j,1..4} of L_h (Proposition 3.1) of every strip:
 * nsub x 4 x ny x ny complex, row-major blocks; blocks a strip does not have
 * (X^{1,1..3}, X^{N,2..4}) are zero.  In the modal form (osm_options.lh_form)
 * the blocks are formed from it, O(ny^3) work per block. */
osm_status osm_get_lh_blocks(osm_handle *h, osm_c64 *blocks_dev);

/* Copy the stored block-Thomas factor: for every line of the packed strip
 * layout the dense inverse of its Schur complement (ny x ny, row-major),
 * complex128 in OSM_FP64 and complex64 in OSM_C32_REFINE; (ncx + nsub) * ny
 * * ny elements.  The factor is twisted: in a strip with nx lines and middle
 * line m = (nx-1)/2, lines i < m hold S_i^{-1} (S_0 = D_0, S_i = D_i -
 * U_{i-1}^T S_{i-1}^{-1} U_{i-1}), lines i > m hold T_i^{-1} (T_{nx-1} =
 * D_{nx-1}, T_i = D_i - U_i T_{i+1}^{-1} U_i^T), line m the inverse of
 * D_m - U_{m-1}^T S_{m-1}^{-1} U_{m-1} - U_m T_{m+1}^{-1} U_m^T. */
osm_status osm_get_factor(osm_handle *h, void *dst_dev);

/* Copy the stored y-line-order factor (osm_strip_order() == 1): strip by
 * strip, y-line a = 0 .. ny-1, the dense inverse (nx_j x nx_j, row-major;
 * complex128 in OSM_FP64, complex64 in OSM_C32_REFINE: the complements are
 * formed and inverted in FP64 either way, the inverses rounded to FP32 for
 * storage in the latter) of that y-line's Schur complement, sum_j ny nx_j^2
 * elements.
 * With A_a the block of y-line a and B_a its coupling to y-line a+1, and
 * middle y-line m = (ny-1)/2: y-lines a < m hold T_a^{-1} (T_0 = A_0, T_a =
 * A_a - B_{a-1}^T T_{a-1}^{-1} B_{a-1}), y-lines a > m hold U_a^{-1} (U_{ny-1}
 * = A_{ny-1}, U_a = A_a - B_a U_{a+1}^{-1} B_a^T), y-line m the inverse of
 * A_m - B_{m-1}^T T_{m-1}^{-1} B_{m-1} - B_m U_{m+1}^{-1} B_m^T.  OSM_ESTATE
 * when the handle keeps no y-line factor or has not factored. */
osm_status osm_get_yfactor(osm_handle *h, void *dst_dev);

/* Kernel timing for measurement: enable = 1 resets the counters and brackets
 * every later launch of the strip-solve kernel with HIP events on the
 * handle's stream; enable = 0 stops.  Both return, in *solve_ms and
 * *solve_launches (either may be NULL), the summed kernel time and the
 * launch count accumulated since the last reset. */
osm_status osm_kernel_timing(osm_handle *h, int32_t enable, double *solve_ms,
                             int64_t *solve_launches);

/* Algorithmic bytes of the strip-solve launches timed since the last reset
 * of osm_kernel_timing (stored inverses read by both sweeps, right-hand
 * side, solution and coupling coefficients of every strip solved; a batched
 * launch counts only the instances it did not skip).  The
 * upper-triangle kernels (osm_solve_shape() >= 4) count n (n + 1) / 2
 * elements per inverse.  Divided by the timed milliseconds it gives the
 * achieved bandwidth of the solve. */
osm_status osm_kernel_work(const osm_handle *h, double *solve_bytes);

/* While osm_kernel_timing is enabled, every update kernel of the factor's
 * symmetric sweep (one per pivot block of 128 and factor step) is also
 * bracketed by HIP events.  Returns the summed kernel time, the launch count
 * and the algorithmic flops of those launches since the last reset (8 real
 * flops per complex multiply-add over the upper 64 x 64 tiles that each pass
 * updates).  Single-instance handles only; the batch factor is not timed. */
osm_status osm_factor_timing(osm_handle *h, double *update_ms, int64_t *update_launches,
                             double *update_flops);

/* Workgroups per strip used by the strip solve: opt->team when given, else
 * the value the autotuner picked at the first factorisation (it times a few
 * solves for every feasible team size).  0 for a NULL handle. */
int32_t osm_solve_team(const osm_handle *h);

/* Kernel and tile shape of the strip solve picked with the team size: 0 .. 3
 * stream full rows of the stored inverses, 4 .. 7 only their upper triangles
 * (waves per workgroup x rows kept in registers as for 0 .. 3).  0 for a
 * NULL handle. */
int32_t osm_solve_shape(const osm_handle *h);

/* Unknown order of the strip factor in use: 0 = node-line order, 1 = y-line
 * order (osm_options.strip_order; with 2 the autotuner's choice, known after
 * the first factorisation, node-line order before it).  0 for a NULL handle. */
int32_t osm_strip_order(const osm_handle *h);

/* How L_h is applied (osm_options.lh_form, Section 4.2): 0 = not built
 * (classical algorithm), 1 = dense blocks per strip class, 2 = modal form by
 * dense real transforms, 3 = modal form by FFT.  0 for a NULL handle. */
int32_t osm_lh_form(const osm_handle *h);

/* ---------------------------------------------------------------- learned guess
 * A network predicts the next step's interface start from the history (the
 * paper starts from the previous converged vector, Section 5; the converged
 * answer does not depend on the start).  Per interface i, along its ny
 * nodes: inputs Re/Im of (r_i, l_{i+1}) of g_{n-1} and g_{n-2}, divided by
 * s_i = rms of g_{n-1}'s two traces (1 if zero), and W_n on the interface
 * line divided by max(1, max|W_n| there): 9 channels.  Outputs (4 channels)
 * are Re/Im of what linear extrapolation misses, g_n - 2 g_{n-1} + g_{n-2},
 * of the two traces divided by s_i; the guess is 2 g_{n-1} - g_{n-2} + s_i y.
 * Network conv1d(9 -> 64, k 5) -> GELU (erf) -> conv1d(64 -> 4, k 5), zero
 * padding; bfloat16 parameters (rounded from an FP32 master copy), FP32
 * accumulation.  Parameters are one FP32 vector of osm_net_nparams() values
 * in the order W1 (64,9,5), b1 (64), W2 (4,64,5), b2 (4).  Tensors x (T,9,L),
 * targets and outputs (T,4,L) are FP32 device arrays, row-major. */

int32_t osm_net_nparams(void);

/* Network with workspace for training batches of up to max_traces traces;
 * parameters zero until osm_net_set_params. */
osm_status osm_net_create(int32_t max_traces, void *hip_stream, osm_net **out);

/* Set the FP32 master parameters (device array) and reset the optimiser. */
osm_status osm_net_set_params(osm_net *net, const float *theta_dev);

/* Copy the master parameters, or (rounded = 1) the bfloat16 values the
 * network computes with, as FP32. */
osm_status osm_net_get_params(const osm_net *net, int32_t rounded, float *theta_dev);

/* y = network(x) for T traces of length L. */
osm_status osm_net_forward(osm_net *net, const float *x_dev, int32_t T, int32_t L,
                           float *y_dev);

/* Mean squared error of network(x) against t over all T*4*L outputs, and its
 * gradient with respect to the (bfloat16) parameters into grad_dev (NULL =
 * keep internal).  loss may be NULL. */
osm_status osm_net_loss_grad(osm_net *net, const float *x_dev, const float *t_dev,
                             int32_t T, int32_t L, float *grad_dev, double *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * master parameters with the gradient of the batch; the bfloat16 copy is
 * refreshed.  *loss (may be NULL, then no synchronisation) is the loss
 * before the update. */
osm_status osm_net_train_step(osm_net *net, const float *x_dev, const float *t_dev,
                              int32_t T, int32_t L, double lr, double *loss);

/* Largest T of osm_net_loss_grad_noalloc. */
#define OSM_NET_NOALLOC_MAX_TRACES 256

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the loss
 * and gradient of osm_net_loss_grad, from the same kernels in the same
 * order of summation, so the same bits, but with the per-trace partials in
 * one static device array per GPU (about 4.3 MB, held until the process
 * ends) instead of the network's workspace.  The call allocates nothing
 * and does not synchronise: it enqueues on the network's stream, on the
 * network's device, and returns.  T may exceed the network's max_traces,
 * up to OSM_NET_NOALLOC_MAX_TRACES (larger T: OSM_EINVAL, nothing
 * enqueued).  grad_dev (required) receives osm_net_nparams() FP32 values;
 * loss_dev (device, may be NULL) the loss as one double.  Every call on
 * one GPU uses the same array: calls that overlap on one GPU (from several
 * host threads or on several streams) race and must be serialised by the
 * caller. */
osm_status osm_net_loss_grad_noalloc(const osm_net *net, const float *x_dev, const float *t_dev,
                                     int32_t T, int32_t L, float *grad_dev, double *loss_dev);

void osm_net_destroy(osm_net *net);
const char *osm_net_last_error(const osm_net *net);

/* Network inputs x (nsub-1, 9, ny) from g1 = g_{n-1}, g2 = g_{n-2} and the
 * handle's W_n; with g0 = g_n also the targets t (nsub-1, 4, ny) (g0_dev and
 * t_dev both NULL or both given).  Used to build training data from the
 * converged vectors of a run. */
osm_status osm_guess_features(osm_handle *h, const osm_c64 *g1_dev, const osm_c64 *g2_dev,
                              const osm_c64 *g0_dev, float *x_dev, float *t_dev);

/* Network used by opt->guess == 2 (the caller keeps it alive; NULL clears). */
osm_status osm_set_guess_net(osm_handle *h, const osm_net *net);

/* ---------------------------------------------------------------- batches
 * nb independent instances (each its own mesh, strip layout, p and
 * potential; Section 2: one problem statement per instance) advanced
 * together with the classical algorithm (eq. fluxlr).  Every time-step kernel
 * covers all instances in one launch; the strip solve takes the strips of
 * all instances from one work queue in a persistent grid; a chunk of Schwarz
 * iterations is captured once as a HIP graph and replayed until every
 * instance meets its own stopping test, so each instance converges exactly
 * as it would alone.  The single-instance entry points return OSM_ESTATE on
 * a batch handle, and the batch entry points on a single handle.
 * osm_kernel_timing works on a batch handle (timed steps then run the chunk
 * launch by launch instead of as a graph). */

/* Footprint of osm_setup_batch.  opt->algo is OSM_CLASSICAL or OSM_PRECOND
 * (Section 3, eq. algo_pd; every instance builds the L_h of its own strip
 * classes, and its preconditioned update runs inside the replayed step with
 * GMRES, krylov = 0); OSM_EUNSUPPORTED for OSM_INTERFACE_KRYLOV, EINVAL for
 * the S_pade^m condition or BiCGStab in a batch. */
osm_status osm_query_batch(const osm_problem *probs, int32_t nb,
                           const osm_options *opt, osm_footprint *out);

/* probs: host array of nb problems (strip_cells read during the call).  One
 * opt for all.  OSM_ENOMEM before any allocation when the summed footprint
 * exceeds free device memory or opt->mem_cap. */
osm_status osm_setup_batch(const osm_problem *probs, int32_t nb,
                           const osm_options *opt, void *hip_stream,
                           osm_handle **out);

/* W_devs: host array of nb device pointers, W_n of each instance (global
 * nodes of that instance).  Factors every instance; the first call also
 * runs the autotuner of the batched solve (tile shape x workgroups per
 * strip, timed on the batch itself). */
osm_status osm_factor_batch(osm_handle *h, const double *const *W_devs);

/* u_devs: host array of nb device pointers, u_{n-1} in and u_n out for every
 * instance.  stats: host array of nb entries (may be NULL).  On OSM_ENOCONV
 * or OSM_ENONFINITE no instance's u is changed and stats hold the
 * iteration counts reached. */
osm_status osm_step_batch(osm_handle *h, osm_c64 *const *u_devs,
                          osm_step_stats *stats);

/* The autotuner's choice: tile-shape index, team rule alpha (0 = one
 * workgroup per strip; else strips costing more than alpha times the mean
 * work per workgroup get proportionally more), grid size (the resident
 * capacity of the chosen shape) and the work items of the whole-batch plan.
 * During a step the items are re-planned, with the same shape and rule,
 * over the instances still iterating.  Any output may be NULL. */
osm_status osm_batch_tuning(const osm_handle *h, int32_t *variant, double *alpha,
                            int32_t *workgroups, int32_t *items);

void osm_destroy(osm_handle *h);
const char *osm_last_error(const osm_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* OSM_H */
