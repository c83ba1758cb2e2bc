/*
 * c4m.h -- C ABI of the MI355X stepper for the compact fourth-order
 * staggered (Yee) scheme of Versano, Turkel and Tsynkov, "Fourth order
 * accurate compact scheme for first-order Maxwell's equations"
 * (arXiv 2306.17263).
 *
 * One call to c4m_step advances the PEC cavity problem by whole time steps.
 * Each step is the paper's Step 1 followed by Step 2 (Section 3.4):
 *   E^{n+1}   = E^n + r Phi_E,       M Phi_E = Z curl^A G(H^{n+1/2})
 *   H^{n+3/2} = H^{n+1/2} + r Phi_H,  M Phi_H = -(1/Z) curl^A (alpha E^{n+1} + l^{n+1}/12)
 * with r = h_tau/h, alpha = 1 + 2/r^2, beta = r^2/24,
 *   M   = alpha I - beta L9    (eq:ell times h_tau^2/24; L9 the 9/19-point
 *                               Singer-Turkel stencil, Definition def:operatorsP),
 *   G u = alpha u + L5 u / 12  (P2 of Definition def:operatorsP, h^2-scaled),
 *   curl^A                     (the Pade curl of Appendix A.1, eq:lhs, times h),
 *   l   = h^2 Delta E          (carried from step to step as printed in Step 1,
 *                               or recomputed as L5 E in the DISCRETE variant).
 * Boundary treatment: tangential E = 0 on the walls (eq:bc_E=0), normal H
 * constant in time (eq:BC_H), even ghosts for the Neumann directions
 * (Corollary cor:ghost_cor).  c4m_step takes J = rho = 0; c4m_step_source
 * steps a 2D (TM) problem driven by a current Jz (Section 3.1).
 *
 * Memory and streams: the caller owns the device workspace (size from
 * c4m_workspace_bytes, 256-byte aligned) and the HIP stream; the library
 * allocates no device memory and keeps only a small host handle.  Device
 * pointers are plain `void*` / `double*` in the current HIP device.
 *
 * Field layout at the ABI: FP64, row-major (nz, ny, nx) with x fastest,
 * walls included.  Component s of E sits at half points along s and nodes
 * along the other axes; component s of H at nodes along s and half points
 * along the others (eq:meshes).  A node axis has N+1 points, a half axis N.
 * In 2D (TM: Ez, Hx, Hy) nz = 1.
 *
 * Errors: every function returns a c4m_status; nothing throws across the
 * ABI.  c4m_last_error() returns a thread-local text for the last failure.
 * Threading: one problem handle must not be used by two threads at once.
 */
#ifndef C4M_H
#define C4M_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    C4M_OK = 0,
    C4M_EINVAL = -1,       /* bad argument, shape or configuration              */
    C4M_ENOMEM = -2,       /* workspace too small                               */
    C4M_EDEVICE = -3,      /* a HIP call failed                                 */
    C4M_ESTATE = -4,       /* call not valid in the handle's state              */
    C4M_ENOCONV = -5,      /* PCG missed its tolerance: reported as c4m_info.noconv *
                            * (sticky); c4m_step does not wait to find out      */
    C4M_EUNSTABLE = -6,    /* CFL number above the paper's stability bound      */
    C4M_ENONFINITE = -7    /* a non-finite value was detected (sticky)          */
} c4m_status;

typedef enum {
    C4M_EX = 0, C4M_EY = 1, C4M_EZ = 2,
    C4M_HX = 3, C4M_HY = 4, C4M_HZ = 5,
    C4M_LX = 6, C4M_LY = 7, C4M_LZ = 8     /* l_s = h^2 (Delta E)_s on E_s's grid */
} c4m_field;

enum { C4M_CLOSURE_PAPER = 0,    /* printed closure rows (26,-5,4,-1)/24 of eq:lhs  */
       C4M_CLOSURE_REFLECT = 1 };/* image closure (23,1)/24 or (22,1)/24            */
enum { C4M_LAP_TRACKED = 0,      /* carry l = h^2 Delta E as in Step 1              */
       C4M_LAP_DISCRETE = 1 };   /* recompute l = L5 E (second-order Laplacian)     */
enum { C4M_FP64 = 0,             /* all arithmetic in FP64                          */
       C4M_FP32_REFINED = 1 };   /* FP32 sweeps, FP64 residuals and state           */
enum { C4M_SCHEME_C4 = 0,        /* the compact fourth-order scheme (Section 3.4)   */
       C4M_SCHEME_NC = 1 };      /* the non-compact comparison scheme NC (Section   *
                                  * 5.2): the Yee update with stencil K4 at a = 0,  *
                                  * one-sided rows at the walls; 2D, FP64, no solve; *
                                  * closure, lap_mode, solver, sweeps ignored;      *
                                  * CFL bound 6/(7 sqrt 2) (leapfrog with K4)       */
enum { C4M_SOLVER_CHEBYSHEV = 0, /* reduction-free Chebyshev on the closed-form     *
                                  * spectral bounds of M (Appendix A.2)             */
       C4M_SOLVER_PCG = 1,       /* Jacobi-preconditioned CG with device dot products */
       C4M_SOLVER_TRANSFORM = 2 }; /* exact: DST-I / DCT-II along each axis (Appendix *
                                  * A.2) as FP64 matrix products; FP64 only         */

#define C4M_FLAG_ALLOW_ANY_CFL 0x1u   /* skip the CFL guard of create               */
#define C4M_FLAG_CHECK_FINITE  0x2u   /* scan the fields for NaN/Inf after each call */
#define C4M_FLAG_PROFILE       0x4u   /* time every launch (group) of a kernel class *
                                       * with HIP events on the problem's stream (no   *
                                       * host waits; c4m_get_info reads them)          */
#define C4M_FLAG_DIRECT        0x8u   /* launch every step directly, never as a     *
                                       * captured graph (for batches whose members   *
                                       * change often, where a capture per new batch *
                                       * would cost more than it saves)               */

/* Kernel classes reported by the profiling counters of c4m_info. */
enum { C4M_K_RHS_E = 0,      /* Pade curl of G(H): Step 1 right-hand side          */
       C4M_K_SOLVE_E = 1,    /* compact solve + E (and G_E) update                 */
       C4M_K_RHS_H = 2,      /* Pade curl of G_E: Step 2 right-hand side           */
       C4M_K_SOLVE_H = 3,    /* compact solve + H update                           */
       C4M_K_STEP_E = 4,     /* fused Step 1 (right-hand side, solve, update)      */
       C4M_K_STEP_H = 5,     /* fused Step 2                                       */
       C4M_K_OTHER = 6,      /* everything else; the source corrections of        *
                              * c4m_step_source (one group per component)        */
       C4M_K_STEP = 7,       /* a whole step in one launch (batched strip form)    */
       C4M_K_COUNT = 8 };

typedef struct {
    int32_t dim;        /* 2 = TM (Ez, Hx, Hy), 3 = full Maxwell                       */
    int32_t n;          /* cells per side, h = 1/n; 8 <= n <= 16384 (2D), 1024 (3D)     */
    double cfl;         /* r = h_tau / h; rejected above 5/(6 sqrt 2) in 2D and         *
                         * 5/(6 sqrt 3) in 3D (Section 4) unless ALLOW_ANY_CFL          */
    double z;           /* impedance Z > 0                                              */
    int32_t closure;    /* C4M_CLOSURE_*                                               */
    int32_t lap_mode;   /* C4M_LAP_*                                                   */
    int32_t precision;  /* C4M_FP64 or C4M_FP32_REFINED                                */
    int32_t solver;     /* C4M_SOLVER_*                                                */
    int32_t sweeps;     /* Chebyshev M-applications per solve (0 = the fewest whose    *
                         * contraction is below 4e-16: 5 at 2D r = 0.5, 4 at 3D r = 0.4) */
    int32_t max_iter;   /* PCG iteration cap per solve (0 = 16)                         */
    double rtol;        /* PCG relative residual target (0 = 1e-14)                    */
    int32_t tile_x;     /* column kernel shape, 0..4 (0 = built-in, see below)         */
    int32_t tile_y;
    uint32_t flags;     /* C4M_FLAG_*                                                  */
    int32_t batch_wait_limit; /* batched strip form: polls before a stage wait gives  *
                               * up and flags (0 = about a second); see c4m_batch_check */
    int32_t scheme;     /* C4M_SCHEME_* (0 = the compact scheme)                       */
    int32_t reserved[3];
} c4m_config;
/* tile_x, single 2D problems (FP64 Chebyshev): 0 = wave strips (one
 * wavefront per 64 columns walks down a row segment, no LDS; falls back
 * to 3 where it does not apply), 4 = wave strips unrolled 16 steps,
 * 1 = 64 x 4 column tiles, 2 = 128 x 2, 3 = 128 x 4.  Batched form:
 * 0 = wave strips (FP64; column tiles 128 x 4 in the FP32-refined form),
 * 1 = 64 x 4 column tiles, 2 = 128 x 2.  3D: ignored.
 * tile_y, batched form: with the strips, 1 = one persistent launch per
 * step, any other value = one persistent launch per stage (default);
 * with column tiles, a multiplier of the persistent grid (0 = 1). */

typedef struct {
    int64_t steps;            /* whole steps taken since create                       */
    double tau_e, tau_h;      /* time of E and of H relative to the initial data      */
    int32_t sweeps;           /* Chebyshev applications per solve in use              */
    int32_t last_iters;       /* PCG: iterations of the last solve                    */
    int32_t max_iters;        /* PCG: most iterations of any solve so far             */
    double last_rel_residual; /* PCG: relative residual of the last solve             */
    int32_t nonfinite;        /* sticky: a NaN/Inf was seen                           */
    int32_t noconv;           /* sticky: a PCG solve hit max_iter                     */
    size_t workspace_bytes;   /* bytes of the caller's workspace in use               */
    /* With C4M_FLAG_PROFILE: summed kernel time (ms) and launch count per
     * C4M_K_* class since create (get_info synchronises the stream). */
    double kernel_ms[C4M_K_COUNT];
    int64_t kernel_launches[C4M_K_COUNT];
    /* Algorithmic HBM bytes per launch of each class: the compulsory FP64
     * state traffic of the scheme (temporaries excluded). */
    double kernel_alg_bytes[C4M_K_COUNT];
} c4m_info;

typedef struct c4m_problem c4m_problem;
typedef struct c4m_batch c4m_batch;

/* Fill *cfg with the defaults: dim 2, n 64, cfl 0.5, z 1, PAPER closure,
 * carried Laplacian, FP64, Chebyshev. */
c4m_status c4m_config_default(c4m_config* cfg);

/* Bytes of device workspace a problem with this configuration needs. */
c4m_status c4m_workspace_bytes(const c4m_config* cfg, size_t* bytes);

/* Create a problem on `d_workspace` (caller-owned, >= c4m_workspace_bytes,
 * 256-byte aligned, on the current device) and `hip_stream` (NULL = the
 * null stream).  Uploads the Pade coefficient tables asynchronously on the
 * stream and zeroes every field.  No kernel runs before this returns except
 * those uploads and fills.  EUNSTABLE when cfl exceeds the paper's bound. */
c4m_status c4m_create(const c4m_config* cfg, void* d_workspace, size_t bytes,
                      void* hip_stream, c4m_problem** out);

/* Stored extent of a field as (nz, ny, nx).  EINVAL for a field the
 * dimension does not have (e.g. C4M_EX in 2D). */
c4m_status c4m_field_shape(const c4m_problem* p, c4m_field f, int64_t shape[3]);

/* Copy a whole field in (E at tau = 0, H at tau = h_tau/2, l at tau = 0).
 * `src` is a device pointer when src_on_device != 0, else host memory.
 * E and l components synchronise the stream (their wall values are checked
 * first); H from host memory too.  Tangential E and l vanish on PEC walls
 * (eq:bc_E=0 and, for l = h^2 Delta E, d^2 E_tan / dt^2 = 0 there): EINVAL,
 * and nothing changed, when a wall value exceeds 1e-13 of the array's
 * largest magnitude; smaller ones (rounding of sampled data) are stored as
 * 0.  The whole array of an H component is taken, walls included: the
 * values on the walls normal to its axis are the constant normal H of
 * eq:BC_H.  If l is never set after E, the library uses l = L5 E. */
c4m_status c4m_set_field(c4m_problem* p, c4m_field f, const double* src, int src_on_device);

/* Wall values of one component on one face (face = 2 axis + side, axis
 * 0..dim-1 for x, y, z, side 0 the wall at coordinate 0, 1 the wall at 1).
 * `vals` is the component's wall plane: its (nz, ny, nx) extent without
 * `axis`, remaining axes in that order, x fastest (host memory, or device
 * memory when vals_on_device != 0; host data synchronise the stream).
 * H_s: only the two faces normal to axis s (the points H_s has on walls);
 * the values are its normal component there, constant in time on a PEC
 * wall (eq:BC_H, Table tab:bc), and enter the source conditioning of
 * Step 1 as the wall values of the node-direction stencil.
 * E_s and l_s: only faces normal to the other axes, and every value must be
 * 0 (tangential E vanishes, eq:bc_E=0): EINVAL otherwise, nothing changed.
 * EINVAL for any other face. */
c4m_status c4m_set_boundary(c4m_problem* p, c4m_field f, int32_t face, const double* vals, int vals_on_device);

/* Copy a whole field out; a host destination synchronises the stream. */
c4m_status c4m_get_field(c4m_problem* p, c4m_field f, double* dst, int dst_on_device);

/* Enqueue nsteps whole steps on the problem's stream (asynchronous);
 * nsteps = 0 does nothing.  Runs of up to 32 steps are captured once each
 * as a HIP graph and replayed (the launch sequence of a step, Section 3.4
 * Step 1 then Step 2); on the null stream, with C4M_FLAG_PROFILE, or while
 * the caller captures the stream, the launches go to the stream directly.  With C4M_FLAG_CHECK_FINITE the call scans the
 * fields afterwards, waits, and returns ENONFINITE (sticky in c4m_info)
 * when a NaN or Inf is found. */
c4m_status c4m_step(c4m_problem* p, int64_t nsteps);

/* Capture, once, the graphs that c4m_step(p, nsteps) replays (runs of up to
 * 32 steps and the remainder), without running anything, so that a later
 * c4m_step with that count only launches them.  Lets a caller build them
 * off its critical path (another thread, a set-up stream).  No-op where
 * c4m_step launches directly (profiling, null stream, capture in progress).
 * EINVAL for nsteps < 0. */
c4m_status c4m_prepare(c4m_problem* p, int64_t nsteps);

/* Move the problem to another HIP stream: waits for the work queued on its
 * current stream, then every later call enqueues on `stream` (graphs
 * captured before stay valid).  For handing a problem set up on a private
 * stream to the stream it will be stepped on.  ESTATE for a batch member. */
c4m_status c4m_set_stream(c4m_problem* p, void* stream);

/* Taylor start (Section 5.1, eq:talorh, J = 0): with E set at tau = 0 and
 * H set at tau = 0 (not yet stepped), replace H by H at tau = h_tau/2:
 *   H + a H_t + a^2/2 H_tt + a^3/6 H_ttt + a^4/24 H_tttt,  a = h_tau/2,
 * H_t = -(1/Z) curl E (the scheme's Pade curl), H_tt = Delta H, H_ttt =
 * Delta H_t, H_tttt = Delta H_tt (the second-order Laplacian Delta_h with
 * the ghost rules of Corollary cor:ghost_cor); H keeps its values on the
 * walls it is normal to.  Asynchronous; ESTATE after a step, EINVAL for the
 * NC scheme. */
c4m_status c4m_init_h_taylor(c4m_problem* p);

/* Sources (Section 3.1: eq:mh, Table tab:spec; Section 3.3: the ghost values
 * of Method 2, eq:gst2), 2D TM problems with a current J = (0, 0, Jz).  The
 * caller supplies J and the derivatives that the scheme's formulas need,
 * sampled at the right times; the library forms the source terms, the ghost
 * values and the solves.  Every pointer is device memory (FP64, dense, x
 * fastest, the layout of c4m_set_field); NULL stands for zeros.  Readings
 * followed (the printed source terms disagree with the derivation that
 * precedes them; the derivation is followed):
 *   Step 1 adds F_J = -Z (Jz + (h_t^2/24) d2Jz/dt2) to F, Step 2 adds
 *   (h_t^2/24) curl dJ/dt; each with its Laplacian as given (the eq:helm2
 *   form); ghosts along a half-point axis phi(-h/2) = phi(h/2) - h q,
 *   q = phi_n + (h^2/24) phi_nnn (eq:gst2), for H in G(H) (Step 1) and for
 *   delta_t H in the rows of M next to the walls (Step 2); on the E walls
 *   G_E = (h^2/12) Z dJz/dt (there Delta Ez = Z dJz/dt). */
typedef struct c4m_source_tm {
    /* Step 1, at tau^{n+1/2}, on the Ez grid ((N+1) x (N+1)) */
    const double* jz;            /* Jz */
    const double* jz_tt;         /* d2 Jz / dtau2 */
    const double* jz_lap;        /* Delta Jz */
    const double* jz_tt_lap;     /* Delta d2 Jz / dtau2 */
    /* H at tau^{n+1/2} on its half-point walls, N+1 values along the wall
     * (node points): hx_wall[w][0] = dHx/dy, hx_wall[w][1] = d3Hx/dy3 at
     * y = w; hy_wall[w][0] = dHy/dx, hy_wall[w][1] = d3Hy/dx3 at x = w */
    const double* hx_wall[2][2];
    const double* hy_wall[2][2];
    /* Step 2, at tau^{n+1} */
    const double* jz_t;          /* dJz/dtau on the Ez grid (read on the walls) */
    const double* kx;            /* (curl dJ/dtau)_x = d/dy dJz/dtau, Hx grid (N x (N+1)) */
    const double* kx_lap;        /* its Laplacian */
    const double* ky;            /* (curl dJ/dtau)_y = -d/dx dJz/dtau, Hy grid ((N+1) x N) */
    const double* ky_lap;
    const double* dhx_wall[2][2];   /* as hx_wall and hy_wall, of dH/dtau */
    const double* dhy_wall[2][2];
} c4m_source_tm;

/* Device bytes of the `work` argument of c4m_step_source (0 for a problem
 * that cannot take sources). */
size_t c4m_source_work_bytes(const c4m_problem* p);

/* One step with sources (asynchronous, on the problem's stream): the step
 * of c4m_step plus, in each half-step, the solve of M for the source part
 * of the right-hand side (M's Chebyshev iteration in FP64, the problem's
 * schedule), added to the field before the next half-step reads it.  `work`:
 * device memory of at least c4m_source_work_bytes(p) bytes, 256-byte
 * aligned, the caller's; the first call with a buffer writes the library's
 * tables into it (an asynchronous copy from host memory), later calls with
 * the same pointer use them as they are, so the caller leaves its contents
 * alone between calls and gives each problem a buffer of its own.  The source arrays and `work` must stay valid until
 * the stream has run the step.  EINVAL unless 2D, the compact scheme and
 * the PAPER closure (the REFLECT rows assume homogeneous Neumann data), or
 * for a short `work`; ESTATE for a batch member.  With C4M_FLAG_CHECK_FINITE
 * the call scans the fields afterwards as c4m_step does. */
c4m_status c4m_step_source(c4m_problem* p, const c4m_source_tm* src, void* work, size_t work_bytes);

/* Counters and sticky flags; synchronises the stream when PCG statistics
 * or the finite check are involved. */
c4m_status c4m_get_info(c4m_problem* p, c4m_info* info);

/* Release the host handle (the workspace stays the caller's). */
c4m_status c4m_destroy(c4m_problem* p);

/* Batched form: `count` independent problems (2D, any mix of n; shared cfl,
 * z, closure, lap_mode, precision; Chebyshev solve only) on one workspace.
 * A step is four stages per problem (Step 1 x-lines, Step 1 solve, Step 2
 * x-lines, Step 2 Hx and Hy solves), each a table of work items over every
 * problem.  Strip form (FP64, tile_x 0, the default): ONE persistent launch
 * per step; an item waits for its own problem's previous stage only
 * (per-problem counters), so stages of different problems overlap; every
 * member's strip segments are planned for its share of the device.  Column
 * tiles (tile_x 1-3, FP32-refined): one persistent launch per stage.  Runs
 * of steps are captured once as HIP graphs and replayed.  Members equal the
 * same problems stepped alone, bit for bit.  EINVAL for 3D problems, mixed
 * settings or the PCG solver. */
c4m_status c4m_batch_workspace_bytes(const c4m_config* cfgs, int32_t count, size_t* bytes);
c4m_status c4m_batch_create(const c4m_config* cfgs, int32_t count, void* d_workspace,
                            size_t bytes, void* hip_stream, c4m_batch** out);
/* Borrow the handle of problem i (owned by the batch; use it for set/get). */
c4m_status c4m_batch_problem(c4m_batch* b, int32_t i, c4m_problem** out);
/* Advance every problem of the batch by nsteps steps (asynchronous). */
c4m_status c4m_batch_step(c4m_batch* b, int64_t nsteps);
/* Synchronise the batch's stream and report whether a stage wait of the
 * strip form gave up since the last check (EDEVICE: the results of the
 * steps in between are invalid; the flag is cleared).  A wait gives up only
 * if the device does not run every workgroup of the launch at once, e.g.
 * when other work occupies it, or with a tiny batch_wait_limit. */
c4m_status c4m_batch_check(c4m_batch* b);
/* Summed member figures (steps, workspace bytes, algorithmic bytes per
 * launch of each kernel class over all members; C4M_K_STEP for the single
 * launch per step) and, with C4M_FLAG_PROFILE in the members' settings,
 * the batch's kernel time per class: every launch is then bracketed by HIP
 * events on the batch's stream and steps run without graphs (synchronises
 * the stream). */
c4m_status c4m_batch_get_info(c4m_batch* b, c4m_info* info);
c4m_status c4m_batch_destroy(c4m_batch* b);

/* Batched form over problems the caller already created (each on its own
 * workspace, sharing cfl, z, closure, lap_mode, precision, solver, sweeps and
 * tiles).  `d_tables` (>= c4m_batch_tables_bytes of the same problems,
 * 256-byte aligned) holds only the work tables; the problems stay the
 * caller's, must outlive the batch, and keep their own stream-ordered state
 * (they are stepped on the batch's stream).  Lets a serving loop re-form
 * batches as requests come and go without moving resident fields.
 * 3D members (any N; FP64 Chebyshev form only, else EINVAL): every launch of
 * the 3D step (Section 3.4, Step 1 and Step 2) runs once over all members,
 * each member's share of the workgroups running the single-problem kernel
 * body, so a member's fields equal those of the problem stepped alone, bit
 * for bit.  c4m_batch_create takes 2D configurations only. */
c4m_status c4m_batch_tables_bytes(c4m_problem* const* probs, int32_t count, size_t* bytes);
c4m_status c4m_batch_create_from(c4m_problem* const* probs, int32_t count, void* d_tables,
                                 size_t bytes, void* hip_stream, c4m_batch** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): advance
 * the fields `fields[f]` (device pointers indexed by c4m_field, in the
 * layout of c4m_set_field; every field the configuration carries must be
 * given, the others are ignored; with the carried Laplacian the l arrays
 * too) by nsteps steps in place.  The problem's workspace (padded fields,
 * G_E, temporaries, tables, counters) is a 64 MiB static device array, one
 * per device, held until the process ends; the call allocates no device
 * memory, runs the same kernels as c4m_create / c4m_set_field / c4m_step /
 * c4m_get_field on a caller workspace (same results, bit for bit), and
 * returns when the fields are written.  ENOMEM for a configuration whose
 * c4m_workspace_bytes exceeds 64 MiB (2D up to n = 1150 or so, 3D up to
 * n = 76), EINVAL with C4M_FLAG_PROFILE, errors of c4m_set_field otherwise.
 * Calls on one device share the array: the library serialises calls of one
 * process on a device; the array keeps the last call's contents, and each
 * call clears what must start at zero. */
c4m_status c4m_step_fields_noalloc(const c4m_config* cfg, double* const* fields, int64_t nsteps,
                                   void* hip_stream);

const char* c4m_status_string(c4m_status s);
const char* c4m_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
