/*
 * place3d.h -- C ABI of the MI355X (gfx950) global-placement hot path of analytical
 * heterogeneous die-to-die 3D placement (arXiv 2403.09070).
 *
 * The library evaluates, for instances placed in the cuboid [0,d_x] x [0,d_y] x [0,d_z] of a
 * two-die stack, the pieces of the unconstrained objective  sum_e W^_e(v) + lambda U^(v)
 * (Eq. analytical-placement, Sec. II-A) and takes one preconditioned Nesterov step on it:
 *
 *   place3d_density     bin density map                       (Sec. IV-A, Eq. density-map-accum)
 *   place3d_field       potential and field of the map        (Sec. III-A, Eqs. 3d-poisson-equation
 *                                                              to possion-sol-force)
 *   place3d_field_force density-penalty gradient by field gather (Sec. III-A, Sec. IV-A backward)
 *   place3d_density_vjp exact adjoint of the density map      (differentiation form)
 *   place3d_wl_value / place3d_wl_vjp  forward value and recomputing backward of the wirelength
 *                       model                                  (differentiation form)
 *   place3d_wl_grad     bistratal WA wirelength, its gradient and the FDA z-gradient
 *                                                             (Eqs. wa-model-approx, wl-obj,
 *                                                              wl-model, fda-grad, fda-normalize;
 *                                                              Sec. IV-B)
 *   place3d_step        one GP iteration: all of the above, the mixed-size preconditioner
 *                       (Eq. improved-precond) and a Nesterov move
 *   place3d_plan_fillers host-side sizing of z-fixed and free fillers (Eqs. filler-vol,
 *                       free-filler-vol), appended by the caller as instances of kind FILLER
 *   place3d_md2d_*      multi-die 2D global placement over three 2D fields (Sec. III-C,
 *                       Eq. 2d-place), built on the calls above
 *
 * Instance kinds (PLACE3D_KIND_*) mark macros, fixed instances, fillers and z-held instances;
 * place3d_problem.options selects the paper's baseline algorithms for comparison (Sec. IV).
 *
 * Conventions (all calls):
 *   - Device pointers unless stated (place3d_plan_fillers takes host arrays).  Coordinates are instance centres in length units,
 *     structure-of-arrays float32 [3][n] (x row, y row, z row).  Maps are float32
 *     [Nz][Ny][Nx], x fastest.  CSR arrays are int32, pins sorted by net,
 *     net_start[n_nets] == n_pins.
 *   - The die depth is derived, d_z = N_z (w_b + h_b)/2 with w_b = d_x/N_x, h_b = d_y/N_y
 *     (Sec. V-A); an instance's centre z decides its die: top iff z > d_z/2.
 *   - Gradients are d(objective)/d(coordinate), not forces.  Fixed instances get 0; z-held
 *     instances get 0 in z inside place3d_step and place3d_gp_init.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the default stream) and
 *     never synchronises, except place3d_create, which reads the netlist back to the host once,
 *     and place3d_read_scalars, which waits for the stream to read the optimiser's scalars.
 *   - The caller owns all device memory (inputs, outputs and the workspace).  The library never
 *     allocates device memory.  Arrays named in place3d_problem must outlive the context.
 *   - Return value: PLACE3D_OK (0) or a negative place3d_status.  Argument checks are
 *     synchronous and run on the host before anything is enqueued; on error nothing is
 *     enqueued.  place3d_last_error() gives a message.  No C++ exception crosses the ABI.
 *   - One context must not be used from two host threads at once.  Calls on one context that
 *     overlap on different streams race on its workspace.
 */
#ifndef PLACE3D_H
#define PLACE3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PLACE3D_ABI_VERSION 2

#if defined(__GNUC__) || defined(__clang__)
#define PLACE3D_API __attribute__((visibility("default")))
#else
#define PLACE3D_API
#endif

typedef enum place3d_status {
  PLACE3D_OK = 0,
  PLACE3D_ERR_ARG = -1,         /* null or misaligned pointer, bad enum value                */
  PLACE3D_ERR_SIZE = -2,        /* sizes out of range or inconsistent (grid, CSR, workspace) */
  PLACE3D_ERR_HIP = -3,         /* a HIP runtime call failed; the HIP code is in last_error  */
  PLACE3D_ERR_NONFINITE = -4,   /* place3d_read_scalars: a GP iteration met a NaN or infinity  */
  PLACE3D_ERR_UNSUPPORTED = -5, /* valid request the library does not implement             */
  PLACE3D_ERR_NETLIST = -6      /* CSR not monotone, pin owner out of range, or a filler
                                   with a pin                                                */
} place3d_status;

/* Arithmetic of the spectral contractions (a4, a5). */
enum { PLACE3D_FP32 = 0,        /* float32 operands on float32 MFMA                          */
       PLACE3D_BF16X3 = 1 };    /* split hi/lo bfloat16 operands, three products, f32 accum  */

/* Density-penalty gradient used by place3d_step. */
enum { PLACE3D_DGRAD_FIELD = 0,   /* the paper's field gather: -omega sum_b vol(D∩b) E_b     */
       PLACE3D_DGRAD_ADJOINT = 1  /* exact adjoint of the density map applied to phi vol(b)  */ };

/* Preconditioner used by place3d_step (Eqs. general-precond and improved-precond). */
enum { PLACE3D_PRECOND_MIXED = 0,     /* max{1,|E_i|+lambda q_i} macros, max{1,lambda q_i} else */
       PLACE3D_PRECOND_EPLACE = 1,    /* |E_i| + lambda q_i                                   */
       PLACE3D_PRECOND_EPLACE3D = 2 };/* lambda q_i                                           */

/* Algorithm options (place3d_problem.options bits): the baselines that the paper's adaptive
 * density accumulation and incremental FDA are measured against (Sec. IV), kept to repeat that
 * comparison on this hardware.  Results agree with the default algorithms within rounding.
 * MACRO_INSTANCE: large instances (movable macros, oversized cells) are scattered into the map
 *   instance-parallel, one thread per instance walking all its bins with global float atomics,
 *   instead of the tile-resident bin-parallel sweep (Sec. IV-A); the map's last bits then depend
 *   on atomic order.  Not available with fillers (create returns PLACE3D_ERR_UNSUPPORTED).
 * FDA_VANILLA: every pin's FDA difference comes from a full re-evaluation of its net's exact
 *   bistratal wirelength with the owner on each die, O(|P_e|^2) per net, instead of the
 *   incremental O(|P_e|) evaluation of Sec. IV-B. */
enum { PLACE3D_OPT_MACRO_INSTANCE = 1, PLACE3D_OPT_FDA_VANILLA = 2 };

/* Instance kind bits (uint8 per instance).
 * FILLER: a dummy filler (density model, Sec. III-A): a movable, cell-sized instance with no pins
 *   that takes part in the density map and moves with the density force, but is left out of the
 *   overflow (its excess and its charge).  It may not also be a macro or fixed, carry a pin, or
 *   be wider than a density tile (create returns PLACE3D_ERR_ARG / PLACE3D_ERR_NETLIST).
 * ZFIXED: the instance's z is held: its z-gradient is zero in both objective parts before
 *   anything uses them (the z-fixed fillers of Sec. III-A; allowed on any movable instance). */
enum { PLACE3D_KIND_MACRO = 1, PLACE3D_KIND_FIXED = 2, PLACE3D_KIND_FILLER = 4, PLACE3D_KIND_ZFIXED = 8 };

/* z-gradient of place3d_wl_vjp. */
enum { PLACE3D_WLZ_FDA = 0,     /* the paper's z-gradient: normalised FDA (Eqs. fda-grad,
                                   fda-normalize) plus alpha d p^_e(z)/dz, as place3d_wl_grad      */
       PLACE3D_WLZ_VALUE = 1 }; /* the derivative of the model's value in z: alpha d p^_e(z)/dz only
                                   (the bistratal part changes with z only by steps)               */

/* Layout of the float64 wirelength metrics written by place3d_wl_grad (device, 16 slots). */
enum {
  PLACE3D_M_WA_BI = 0,     /* sum_e of the smoothed bistratal wirelength (x + y)            */
  PLACE3D_M_WA_Z = 1,      /* alpha * sum_e WA p_e(z)                                       */
  PLACE3D_M_HPWL = 2,      /* sum_e exact bistratal = minimal D2D HPWL, HBT optimally placed */
  PLACE3D_M_HPWL3D = 3,    /* sum_e p_e(x) + p_e(y) + alpha p_e(z)  (Def. 3d-hpwl)          */
  PLACE3D_M_NCUT = 4,      /* number of nets with pins on both dies (= #HBT)                */
  PLACE3D_M_NORM_X = 5,    /* |grad_x W^_Bi|_1 over movable instances                       */
  PLACE3D_M_NORM_Y = 6,    /* |grad_y W^_Bi|_1                                              */
  PLACE3D_M_NORM_FDA = 7,  /* |FDA z-gradient|_1 before normalisation                       */
  PLACE3D_M_FDA_SCALE = 8, /* (NORM_X + NORM_Y) / (2 NORM_FDA), 0 if NORM_FDA == 0          */
  PLACE3D_NMETRICS = 16
};

/* Layout of the float64 optimiser scalars in place3d_state.scalars (device, 32 slots). */
enum {
  PLACE3D_S_A = 0,         /* Nesterov a_k                                                  */
  PLACE3D_S_LAMBDA = 1,    /* density weight lambda_k                                       */
  PLACE3D_S_STEP = 2,      /* step size of the last iteration                               */
  PLACE3D_S_ITER = 3,      /* iterations taken                                              */
  PLACE3D_S_OVFL_BOT = 4,  /* per-die overflow at the last evaluation point                 */
  PLACE3D_S_OVFL_TOP = 5,
  PLACE3D_S_ENERGY = 6,    /* 1/2 sum_b rho_b phi_b vol(b) (adjoint form only, else 0)      */
  PLACE3D_S_NONFINITE = 7, /* 0, or 1 + the index of the first iteration (0 = place3d_gp_init's
                              evaluation) whose float64 reductions held a NaN or infinity: step
                              and gradient-change norms, lambda, wirelength totals and norms,
                              overflow excess, energy.  Sticky; place3d_read_scalars checks it */
  PLACE3D_S_WL = 8,        /* slots 8..23: the PLACE3D_M_* metrics at the evaluation point  */
  PLACE3D_NSCALARS = 32
};

/* Stages timed by the optional profiler (place3d_profile_enable / place3d_profile_read). */
enum {
  PLACE3D_STAGE_DENSITY = 0,   /* density map by tiles: fixed-map copy, cell and macro deposits  */
  PLACE3D_STAGE_GEMM = 1,      /* every DCT contraction launch (k_gemm_f32, k_gemm_bf16x3, k_sgemm) */
  PLACE3D_STAGE_ZMIX = 2,      /* z mixing, spectral scaling, x fold / unfold between contractions */
  PLACE3D_STAGE_DGRAD = 3,     /* density gradient: field gather or exact adjoint                */
  PLACE3D_STAGE_WL_NETS = 4,   /* per-net WA / bistratal / FDA kernel                            */
  PLACE3D_STAGE_WL_NODES = 5,  /* per-instance gather of pin shares and z normalisation          */
  PLACE3D_STAGE_UPDATE = 6,    /* preconditioning, Nesterov move, reductions                     */
  PLACE3D_STAGE_BUCKET = 7,    /* bucketing of the cells by density tile (count, scans, scatter) */
  PLACE3D_NSTAGES = 8
};

typedef struct place3d_problem {
  int32_t n_inst;          /* instances: movable cells and macros, fixed instances           */
  int32_t n_pins;
  int32_t n_nets;          /* each count at most 2^28 (PLACE3D_ERR_SIZE beyond): the kernels
                              index [4][n] arrays with 32-bit integers                       */
  int32_t nx, ny, nz;      /* bin grid; nx, ny in [2, 8192]; nz even, in [2, 16]; and at most
                              40,704 density tiles (32 x 32 bins for nz <= 4; 16 x 16 for
                              nz = 16): e.g. 6400 x 6400 at nz = 4 (else PLACE3D_ERR_SIZE)       */
  double die_x, die_y;     /* die extent d_x, d_y (> 0)                                      */
  double gamma;            /* WA smoothing, length units (> 0)                               */
  double alpha;            /* weight of the cut term alpha p_e(z) (>= 0)                     */
  double target_density;   /* rho_t of the overflow metric                                    */
  double lambda_ramp;      /* lambda_{k+1} = lambda_ramp * lambda_k in place3d_step          */
  int32_t precision;       /* PLACE3D_FP32 or PLACE3D_BF16X3                                 */
  int32_t dgrad;           /* PLACE3D_DGRAD_FIELD or PLACE3D_DGRAD_ADJOINT                   */
  int32_t precond;         /* PLACE3D_PRECOND_*                                              */
  int32_t options;         /* PLACE3D_OPT_* bits; 0 for the default algorithms                */
  /* device arrays, caller-owned, read-only, must outlive the context */
  const float* size;       /* float32 [4][n_inst]: w_bot, h_bot, w_top, h_top (Eq. std-size-tech) */
  const uint8_t* kind;     /* uint8 [n_inst], PLACE3D_KIND_* bits                             */
  const int32_t* net_start;/* int32 [n_nets+1]                                                */
  const int32_t* pin2node; /* int32 [n_pins], owner instance of each pin; an instance may own
                              several pins of one net (its FDA difference, Eq. fda-grad, then
                              moves all of them and counts once for that net)                 */
  const float* pin_off;    /* float32 [4][n_pins]: ox_bot, oy_bot, ox_top, oy_top offsets from
                              the owner's centre on each die                                  */
  const float* fixed_xyz;  /* float32 [3][n_inst]: positions used for the fixed instances'
                              constant density map (built once in place3d_create); entries of
                              movable instances are ignored                                   */
} place3d_problem;

typedef struct place3d_state {
  float* u;        /* float32 [3][n_inst] Nesterov major sequence                            */
  float* v;        /* float32 [3][n_inst] evaluation point (the placement)                   */
  float* v_prev;   /* float32 [3][n_inst] previous evaluation point                          */
  float* g_prev;   /* float32 [3][n_inst] preconditioned gradient at v_prev                  */
  double* scalars; /* float64 [PLACE3D_NSCALARS], PLACE3D_S_* slots                          */
} place3d_state;

typedef struct place3d_ctx place3d_ctx;

/* ABI version of the loaded library (PLACE3D_ABI_VERSION it was built with). */
PLACE3D_API int32_t place3d_abi_version(void);

/* Message of the last error on `ctx` (or of the last failed place3d_create when ctx is NULL).
 * The string is owned by the library and valid until the next call on the same context. */
PLACE3D_API const char* place3d_last_error(const place3d_ctx* ctx);

/* Bytes of device workspace a context for `prob` needs (256-byte aligned base required).
 * Holds the DCT bases, intermediate maps, the fixed-instance map, the static net schedule,
 * the node->pin CSR, per-pin partial results and reduction slots. */
PLACE3D_API int32_t place3d_workspace_size(const place3d_problem* prob, size_t* bytes);

/* Validate `prob`, copy the netlist topology to the host once to build the static net
 * schedule and node->pin CSR, fill the workspace (bases, schedule, fixed-instance density map)
 * on `stream`, and return a context.  Synchronises `stream`.  `d_workspace` (device, at least
 * place3d_workspace_size bytes, 256-byte aligned) is owned by the caller and must outlive
 * the context. */
PLACE3D_API int32_t place3d_create(const place3d_problem* prob, void* d_workspace, size_t bytes, void* stream,
                       place3d_ctx** out);

/* Release the host-side context (device memory stays with the caller).  NULL is a no-op. */
PLACE3D_API int32_t place3d_destroy(place3d_ctx* ctx);

/* rho[Nz][Ny][Nx] = fixed-instance map + movable instances at `xyz` (Eq. density-map-accum with
 * the local-smoothness stretch and weight of Sec. IV-A, per-die cell sizes of Eq. std-size-tech
 * and the macro size transition of Eq. macro-size-tech).  `xyz` float32 [3][n_inst]. */
PLACE3D_API int32_t place3d_density(place3d_ctx* ctx, const float* xyz, float* rho, void* stream);

/* Potential and field of `rho` on the bin centres (Eqs. poisson-sol-potential and
 * possion-sol-force, Neumann boundary, zero-mean potential).  Any of phi, ex, ey, ez may be
 * NULL and its transforms are skipped.  `energy` (device float64, may be NULL) receives
 * 1/2 sum_b rho_b phi_b vol(b) and needs phi != NULL.  The map operator rho -> phi is
 * symmetric, so the adjoint of the phi output is the same call. */
PLACE3D_API int32_t place3d_field(place3d_ctx* ctx, const float* rho, float* phi, float* ex, float* ey,
                      float* ez, double* energy, void* stream);

/* Density-penalty gradient by the field gather: grad[a][i] (+)= -lambda omega_i
 * sum_b vol(D_i ∩ b) E_a[b], a = x, y, z.  `accumulate` != 0 adds to grad_xyz. */
PLACE3D_API int32_t place3d_field_force(place3d_ctx* ctx, const float* xyz, const float* ex, const float* ey,
                            const float* ez, float lambda, float* grad_xyz, int32_t accumulate,
                            void* stream);

/* Exact adjoint of place3d_density: grad[a][i] (+)= s sum_b g_rho[b] d rho_b / d v_{a,i},
 * s = scale * (d_scale ? d_scale[0] : 1), including the z-dependence of the macro size
 * transition.  `d_scale` (device float64, one value, may be NULL) carries a factor that lives on
 * the device, such as the incoming gradient of a backward pass; with g_rho = phi, scale = vol(b)
 * it gives the gradient of the energy 1/2 sum_b rho_b phi_b vol(b) (the map rho -> phi is
 * symmetric).  The density is piecewise linear in each coordinate; at a kink the derivative is
 * one-sided: from above, or from below along an axis whose upper edge reaches the region's upper
 * face, which at the bounds of the movable range (z = d_z/4 and 3 d_z/4, a macro against a die
 * side) is the direction the clamp allows.  A z within 2^-20 d_z of a bound counts as on it. */
PLACE3D_API int32_t place3d_density_vjp(place3d_ctx* ctx, const float* xyz, const float* g_rho, float scale,
                                        const double* d_scale, float* grad_xyz, int32_t accumulate, void* stream);

/* Wirelength model at `xyz`: grad[x], grad[y] (+)= gradient of the smoothed bistratal
 * wirelength; grad[z] (+)= normalised FDA gradient (Eqs. fda-grad, fda-normalize) plus
 * alpha d p^_e(z)/dz.  `metrics` (device float64 [PLACE3D_NMETRICS], may be NULL) receives
 * the PLACE3D_M_* values. */
PLACE3D_API int32_t place3d_wl_grad(place3d_ctx* ctx, const float* xyz, float* grad_xyz, double* metrics,
                        int32_t accumulate, void* stream);

/* The wirelength model's value at `xyz` without its gradient (the forward pass of the
 * differentiation form; nothing per pin is stored): metrics (device float64 [PLACE3D_NMETRICS])
 * receives PLACE3D_M_WA_BI .. PLACE3D_M_NCUT, the other slots 0.  In the precision form
 * (precision == PLACE3D_BF16X3) the exponential sums are compensated float32 sums, as in every
 * wirelength call of that form. */
PLACE3D_API int32_t place3d_wl_value(place3d_ctx* ctx, const float* xyz, double* metrics, void* stream);

/* place3d_wl_value for callers that cannot allocate device memory or take workspace scratch
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same metrics, with the call's scratch -- the packed positions and one float64
 * partial per wirelength workgroup and net total -- in a static device array of the library
 * (42 MiB on every GPU the library runs on, held until the process ends; its device address is
 * looked up once per device, by place3d_create or the first call on that device) instead of the
 * context's workspace.  It calls no allocating routine.  Limits: at most 2,097,152 instances and
 * 262,144 wirelength workgroups (PLACE3D_ERR_SIZE beyond, nothing enqueued).  Every call on one
 * GPU shares that array: calls that overlap on one GPU (other streams, other contexts, other host
 * threads) race on it; calls ordered on one stream do not.  Nothing in it needs clearing: each
 * call writes every word it reads first. */
PLACE3D_API int32_t place3d_wl_value_static(place3d_ctx* ctx, const float* xyz, double* metrics, void* stream);

/* Backward pass of the wirelength model: every net's extremes and shifted exponential sums are
 * recomputed from `xyz` (none is kept from the forward pass), and grad (+)= s * dW/dxyz with
 * s = d_scale ? d_scale[0] : 1 (device float64, the incoming gradient) and W = sum_e (W^_e(x) +
 * W^_e(y) + alpha p^_e(z)).  `z_mode` picks the z part: PLACE3D_WLZ_FDA (the paper's surrogate,
 * as place3d_wl_grad) or PLACE3D_WLZ_VALUE (the derivative of W itself).  The workspace holds
 * 16 bytes per pin while the call runs, to sum each instance's pin shares in a fixed order. */
PLACE3D_API int32_t place3d_wl_vjp(place3d_ctx* ctx, const float* xyz, const double* d_scale, int32_t z_mode,
                                   float* grad_xyz, int32_t accumulate, void* stream);

/* Start a GP run from `xyz0` (float32 [3][n_inst]): u = v = clamp(xyz0), lambda_0 =
 * |grad W|_1 / |grad U|_1, the bootstrap point v_prev and its preconditioned gradient g_prev;
 * a = 1, iteration 0. */
PLACE3D_API int32_t place3d_gp_init(place3d_ctx* ctx, place3d_state* state, const float* xyz0, void* stream);

/* One GP iteration at state->v: density, field, wirelength, preconditioned gradient, Lipschitz
 * step, Nesterov move, clamp, lambda *= lambda_ramp; metrics of the evaluation point go to
 * state->scalars. */
PLACE3D_API int32_t place3d_step(place3d_ctx* ctx, place3d_state* state, void* stream);

/* Copy state->scalars (PLACE3D_NSCALARS float64) to the HOST array `host_scalars`, waiting for
 * `stream`: the convergence check of a GP loop.  Returns PLACE3D_ERR_NONFINITE (with the
 * iteration in place3d_last_error) when PLACE3D_S_NONFINITE is set; the scalars are copied
 * either way. */
PLACE3D_API int32_t place3d_read_scalars(place3d_ctx* ctx, const place3d_state* state, double* host_scalars,
                                         void* stream);

/* Filler plan (density model, Sec. III-A, Eqs. filler-vol and free-filler-vol): how many fillers
 * of which square footprint fill the region, for the caller to append as instances (kind
 * FILLER|ZFIXED for the z-fixed ones, at z = 3 d_z/4 on top and d_z/4 below; FILLER for the free
 * ones).  vol_top = 1/2 d_x d_y d_z (1 - u_top), vol_bot = 1/2 d_x d_y d_z (1 - u_bot),
 * vol_free = max{d_x d_y d_z - (vol_top + vol_bot + vol_a), 0}, vol_a = the volume of all
 * instances at the size their z0 gives, d_z = nz (d_x/nx + d_y/ny)/2.  Footprints (the paper
 * gives none): the z-fixed fillers of a die take the mean footprint area of the movable standard
 * cells (kind 0) at that die's size, the free fillers the mean of the two areas; a count is the
 * volume over one filler's volume (area x d_z/2) rounded to nearest, halves up.
 * Host-only arithmetic on HOST arrays: size float32 [4][n_inst] (the problem's layout), kind uint8
 * [n_inst], z0 float32 [n_inst].  Errors: PLACE3D_ERR_ARG for a null pointer, u outside [0, 1] or
 * no movable standard cell; PLACE3D_ERR_SIZE for a bad count or grid. */
typedef struct place3d_filler_plan {
  int64_t n_top, n_bot, n_free;            /* z-fixed top, z-fixed bottom and free filler counts */
  double side_top, side_bot, side_free;    /* square footprint sides                            */
  double vol_top, vol_bot, vol_free, vol_a;
} place3d_filler_plan;

PLACE3D_API int32_t place3d_plan_fillers(int32_t n_inst, const float* size, const uint8_t* kind, const float* z0,
                                         double die_x, double die_y, int32_t nx, int32_t ny, int32_t nz,
                                         double u_top, double u_bot, place3d_filler_plan* out);

/* Profiling.  `on` is a bit mask of stages (bit k = PLACE3D_STAGE_* k; PLACE3D_PROFILE_ALL for
 * every stage, 0 to stop): every later kernel launch of `ctx` in a selected stage is bracketed by
 * a pair of HIP events recorded on the launch stream; place3d_profile_read waits for the recorded
 * events and returns, for `stage`, the summed GPU milliseconds and the number of launches since
 * the last reset (`reset` != 0 clears all stages after reading).  Event objects are host-runtime
 * objects; no device memory is allocated.  Each bracketed launch pays a small overhead, and the
 * events change how launches on the two streams overlap, so a narrow mask perturbs least. */
#define PLACE3D_PROFILE_ALL 0xFF
PLACE3D_API int32_t place3d_profile_enable(place3d_ctx* ctx, int32_t on);
PLACE3D_API int32_t place3d_profile_read(place3d_ctx* ctx, int32_t stage, double* ms, int64_t* launches,
                                         int32_t reset);

/* ------------------------------------------------------------------------------------------
 * Multi-die 2D global placement (Sec. III-C, Eq. 2d-place).  With the die of every instance fixed
 * by a 3D placement, the z axis is dropped: the bottom die, the top die and the layer of hybrid
 * bonding terminals (HBTs) are three independent 2D electrostatic systems with their own weights,
 * and the objective over the planar positions of all nodes is
 *     sum_e W^_e(x, y) + lambda_bot U_bot + lambda_top U_top + lambda_hbt U_hbt,
 * W^_e the WA model (Eq. wa-model-approx) of every partial net: a net with pins on both dies is
 * split into a top and a bottom partial net that share one movable HBT node (the caller builds the
 * nodes and partial nets; the HBTs are nodes of the HBT layer).  Each layer's density, potential,
 * field and field-gather gradient are the 2D forms of place3d_density, place3d_field and
 * place3d_field_force on that layer's nodes; the optimiser is place3d_step's in x and y, with the
 * preconditioner of Eq. improved-precond taken with the node's layer weight and q = w h, lambda_0
 * = |grad W|_1 / |grad U_L|_1 over each layer's movable nodes and all three weights multiplied by
 * lambda_ramp every step.  Overflow of a layer: sum_b max(rho_b - rho_t, 0) area(b) over the map
 * without fillers, divided by the area of its movable non-filler nodes.
 * Conventions as above; positions are float32 [2][n_nodes] (x row, y row). */

enum { PLACE3D_LAYER_BOTTOM = 0, PLACE3D_LAYER_TOP = 1, PLACE3D_LAYER_HBT = 2 };

typedef struct place3d_md2d_problem {
  int32_t n_nodes;         /* instances, HBTs and fillers                                     */
  int32_t n_layer[3];      /* nodes on each layer (must match `layer`; each >= 1)             */
  int32_t n_pins, n_nets;  /* partial nets                                                   */
  int32_t nx, ny;          /* bin grid of every layer; nx, ny in [2, 8192]                   */
  double die_x, die_y;
  double gamma;            /* WA smoothing, length units (> 0)                               */
  double target_density;   /* rho_t of the overflow metric                                    */
  double lambda_ramp;
  int32_t precision;       /* PLACE3D_FP32 or PLACE3D_BF16X3: the three spectral solves       */
  /* device arrays, caller-owned, read-only, must outlive the context */
  const float* size;       /* float32 [2][n_nodes]: w, h on the node's layer                  */
  const uint8_t* kind;     /* uint8 [n_nodes]: PLACE3D_KIND_MACRO, _FIXED, _FILLER bits        */
  const uint8_t* layer;    /* uint8 [n_nodes]: PLACE3D_LAYER_*                                */
  const int32_t* net_start;/* int32 [n_nets+1], partial nets                                  */
  const int32_t* pin2node; /* int32 [n_pins]                                                  */
  const float* pin_off;    /* float32 [2][n_pins]: offset from the owner's centre             */
  const float* fixed_xy;   /* float32 [2][n_nodes]: positions of the fixed nodes              */
} place3d_md2d_problem;

/* Metrics of a multi-die 2D evaluation (device float64 [PLACE3D_NMETRICS]). */
enum { PLACE3D_MD_WA = 0,        /* sum of the partial nets' WA wirelength, x + y            */
       PLACE3D_MD_HPWL = 1,      /* sum of their exact HPWL                                  */
       PLACE3D_MD_OVFL = 2,      /* slots 2, 3, 4: overflow of the bottom, top and HBT layer */
       PLACE3D_MD_ENERGY = 5 };  /* slots 5, 6, 7: U of each layer (place3d_md2d_eval only)   */

/* Optimiser scalars of a multi-die 2D state (device float64 [PLACE3D_NSCALARS]). */
enum { PLACE3D_MS_A = 0,         /* Nesterov a_k                                             */
       PLACE3D_MS_LAMBDA = 1,    /* slots 1, 2, 3: lambda of the bottom, top and HBT layer   */
       PLACE3D_MS_STEP = 4, PLACE3D_MS_ITER = 5,
       PLACE3D_MS_METRICS = 8,   /* slots 8..12: PLACE3D_MD_WA .. OVFL+2 at the evaluation point */
       PLACE3D_MS_NONFINITE = 16 /* as PLACE3D_S_NONFINITE                                    */ };

typedef struct place3d_md2d_state {
  float* u;        /* float32 [2][n_nodes] */
  float* v;
  float* v_prev;
  float* g_prev;
  double* scalars; /* float64 [PLACE3D_NSCALARS], PLACE3D_MS_* slots */
} place3d_md2d_state;

typedef struct place3d_md2d_ctx place3d_md2d_ctx;

/* Workspace bytes (256-byte aligned base) of a multi-die 2D context. */
PLACE3D_API int32_t place3d_md2d_workspace_size(const place3d_md2d_problem* prob, size_t* bytes);
/* Validate, read the node arrays and netlist back once, build the per-layer and wirelength
 * sub-problems in the workspace and create their contexts.  Synchronises `stream`. */
PLACE3D_API int32_t place3d_md2d_create(const place3d_md2d_problem* prob, void* d_workspace, size_t bytes,
                                        void* stream, place3d_md2d_ctx** out);
PLACE3D_API int32_t place3d_md2d_destroy(place3d_md2d_ctx* ctx);
PLACE3D_API const char* place3d_md2d_last_error(const place3d_md2d_ctx* ctx);
/* The objective's parts at `xy`: grad_wl (+)= dW/dxy, grad_den = d U_L / dxy of every node for its
 * own layer L (field gather, not scaled by lambda; zero for fixed nodes), both float32
 * [2][n_nodes]; rho (may be NULL) the three layer maps float32 [3][ny][nx]; metrics (may be NULL)
 * the PLACE3D_MD_* values. */
PLACE3D_API int32_t place3d_md2d_eval(place3d_md2d_ctx* ctx, const float* xy, float* grad_wl, float* grad_den,
                                      float* rho, double* metrics, void* stream);
/* u = v = clamp(xy0), lambda_0 of each layer, the bootstrap point and its gradient. */
PLACE3D_API int32_t place3d_md2d_gp_init(place3d_md2d_ctx* ctx, place3d_md2d_state* state, const float* xy0,
                                         void* stream);
/* One iteration: both objective parts at state->v, the preconditioned gradient, the Lipschitz
 * step, the Nesterov move and the clamp; the three lambdas grow by lambda_ramp. */
PLACE3D_API int32_t place3d_md2d_step(place3d_md2d_ctx* ctx, place3d_md2d_state* state, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PLACE3D_H */
