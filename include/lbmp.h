/*
 * lbmp.h -- C ABI of the MI355X (gfx950) improved MRT pseudopotential
 * lattice Boltzmann library (liblbmp.so).
 *
 * Method: Q. Li, K. H. Luo, X. J. Li, "Lattice Boltzmann modeling of
 * multiphase flows at large density ratio with an improved pseudopotential
 * model" (arXiv:1211.6932).  One time step of the D2Q9 update is
 *   1. pull streaming of the post-collision distributions      Eq. (5)
 *      (x periodic; y periodic or halfway bounce-back walls)    Sec. IV.C
 *   2. density summation                                        Eq. (6)
 *   3. Carnahan-Starling pressure and pseudopotential psi       Eqs. (30), (24)
 *      (or the Sbragaglia-Shan psi of Eq. (23), see lb_psi_form)
 *   4. 8-neighbour interaction force, w(1)=1/3, w(2)=1/12       Eq. (7)
 *   5. half-force-corrected velocity                            Eq. (6)
 *   6. MRT collision in moment space with the improved forcing  Eqs. (2)-(4), (25)
 *      and a density-dependent shear rate (nu_l / nu_g)         Sec. IV.C
 *
 * Conventions common to every entry point
 *   - All calls return lb_status; none throws or aborts.  On failure
 *     lb_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread).
 *   - Device pointers are HIP device addresses (for example a torch tensor's
 *     data_ptr() on a ROCm device).  The caller owns every device buffer:
 *     the workspace, inputs and outputs.  The library owns only the small
 *     host-side context and its captured graphs; lb_destroy frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream, on which step loops are launched without graph capture).
 *     Calls are asynchronous on that stream unless stated otherwise.
 *   - Fields are FP32, row-major [ny][nx], x fastest, contiguous.
 *   - Lattice units throughout: c = dt = 1, c_s^2 = 1/3.
 */
#ifndef LBMP_H
#define LBMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,     /* invalid argument or parameter; nothing was launched          */
    LB_ENOMEM = -2,     /* workspace too small                                           */
    LB_EHIP = -3,       /* a HIP runtime call failed; see lb_last_error()                */
    LB_EUNSTABLE = -4,  /* a site had a non-finite density, b rho/4 >= 1 or psi^2 <= 0
                           (Eq. (24)), or a non-positive density (Eq. (23))              */
    LB_ESTATE = -5      /* context poisoned by an earlier LB_EUNSTABLE / LB_EHIP          */
} lb_status;

typedef enum {
    LB_BC_PERIODIC = 0, /* periodic in x and y                                           */
    LB_BC_WALLS_Y = 1   /* periodic in x; no-slip walls half a cell below row 0 and half
                           a cell above row ny-1 (halfway bounce-back).  psi beyond a
                           wall equals psi of the adjacent fluid row, same column.       */
} lb_bc;

typedef enum {
    LB_STORE_F32 = 0,          /* distributions stored as FP32 (72 B/site/step moved)       */
    LB_STORE_F16_OFFSET = 1,   /* FP16 of f_a - w_a rho_ref, one reference density for the
                                  whole lattice (36 B/site/step)                             */
    LB_STORE_BF16_OFFSET = 2,  /* BF16 of f_a - w_a rho_ref (36 B/site/step)                  */
    LB_STORE_F16_LOCAL = 3,    /* FP16 of f_a - w_a rho(x) with the site's own density
                                  rho(x) stored in FP32 beside them (44 B/site/step)         */
    LB_STORE_BF16_LOCAL = 4,   /* BF16 of f_a - w_a rho(x), rho(x) in FP32 (44 B/site/step)   */
    LB_STORE_F16_DEST = 5      /* FP16 of f*_a(x) / rhohat(x + e_a) - w_a, scaled by the density
                                  of the site that pulls the value (x itself for a population
                                  reflected at a wall); rhohat = bf16 of each site's density,
                                  stored beside it (40 B/site/step)                          */
} lb_store;
/* w_a are the D2Q9 lattice weights 4/9 (rest), 1/9 (axis), 1/36 (diagonal).
 * Collision and force are computed in FP32 for every storage type. */

typedef enum {
    LB_PSI_CS = 0,  /* Eq. (24): psi = sqrt(2 (p_EOS - rho/3) / G) with the Carnahan-Starling
                       p_EOS of Eq. (30) (the paper's choice)                          */
    LB_PSI_SS = 1   /* Eq. (23), Sbragaglia-Shan: psi = exp(-1/rho) for psi_eps = 0, else
                       (rho / (psi_eps + rho))^(1/psi_eps); a, b, R, T are unused and the
                       bulk pressure is rho/3 + G psi^2 / 2.  With sigma = -psi_eps/(16 G)
                       the improved forcing gives epsilon = psi_eps in Eq. (29), so the
                       coexistence densities follow the Maxwell construction (Eq. (22)) of
                       that pressure.                                                   */
} lb_psi_form;

typedef enum {
    LB_STENCIL_NEAREST = 0,    /* Eq. (7) over the eight nearest neighbours, w(1) = 1/3,
                                  w(2) = 1/12 (the paper's stencil)                           */
    LB_STENCIL_MULTIRANGE = 1  /* nearest and next-nearest neighbours (Sec. III.B): the 24 sites
                                  with |e|^2 in {1, 2, 4, 5, 8}, w = 4/21, 4/45, 1/60, 2/315,
                                  1/5040, the weights isotropic to eighth order with
                                  sum w e_x^2 = 1 (the bulk term G psi^2 / 2 is unchanged).
                                  With sigma = 0 a flat interface follows Eq. (21) at
                                  epsilon = 10/31, the value Sec. III.B quotes for such
                                  interactions.  FP32 storage and single lattices only.      */
} lb_stencil;

/* Run parameters.  Rates are the inverse relaxation times 1/tau of Eq. (2).
 * The shear rate is per site: s_nu = 1/(3 nu + 1/2) with nu = nu_l where
 * rho >= rho_switch and nu_g elsewhere (Sec. IV.C; Eq. (10) gives
 * nu = (tau_nu - 1/2)/3).  s_rho and s_j are validated but, with the
 * half-force velocity of Eq. (6), do not change the result (the density and
 * momentum moments after collision are rho and rho v + F/2 for any rate). */
typedef struct {
    int32_t nx, ny;          /* grid size, each >= 3                                     */
    int32_t bc;              /* lb_bc                                                    */
    int32_t store;           /* lb_store                                                 */
    double a, b, R, T;       /* Carnahan-Starling constants and absolute temperature,
                                Eq. (30); b > 0, T > 0, R > 0, a >= 0 (LB_PSI_CS)        */
    double G;                /* interaction strength of Eq. (7), G < 0                   */
    double sigma;            /* improved-forcing coefficient of Eq. (25), >= 0           */
    double s_rho, s_e, s_zeta, s_j, s_q;   /* rates in (0, 2)                            */
    double nu_l, nu_g;       /* kinematic viscosities, > 0                               */
    double rho_switch;       /* density at which nu switches from nu_g to nu_l           */
    double rho_ref;          /* reference density of LB_STORE_*_OFFSET (ignored otherwise) */
    int32_t psi_form;        /* lb_psi_form: pseudopotential of Eq. (24) or of Eq. (23)    */
    int32_t stencil;         /* lb_stencil: interaction stencil of Eq. (7)               */
    double psi_eps;          /* epsilon of Eq. (23), >= 0 (LB_PSI_SS only)               */
} lb_params;

/* An annulus r_min <= d < r_max around (cx, cy); d uses the minimum image in
 * x, and in y when bc is periodic.  r_max may be +inf. */
typedef struct {
    double cx, cy, r_min, r_max;
} lb_region;

/* Reductions over the current state, accumulated in FP64 on the GPU in a
 * fixed order (bitwise reproducible for a given grid and launch shape). */
typedef struct {
    double mass;             /* sum of rho                                               */
    double mom_x, mom_y;     /* sum of rho v, v the half-force velocity of Eq. (6)       */
    double p_in, p_out, dp;  /* mean p_EOS (Eq. 30) over region `in`, `out`, difference  */
    double rho_in, rho_out;  /* mean rho over the two regions                            */
    double n_in, n_out;      /* number of sites in each region                           */
    double max_u;            /* max |v|                                                  */
    int32_t unstable;        /* nonzero if a step since init saw an unstable site        */
    int32_t reserved;
    int64_t step;            /* time t of the state                                      */
} lb_diag;

typedef struct lb_ctx lb_ctx; /* opaque host-side context */

/* Pure host check of the parameter block (no GPU needed).  LB_OK or LB_EINVAL. */
lb_status lb_validate_params(const lb_params* p);

/* Bytes of device workspace lb_init needs for these parameters (0 if invalid).
 * Pure host function. */
size_t lb_workspace_bytes(const lb_params* p);

/* Bytes of one stored state, the size of the buffers lb_get_state /
 * lb_set_state copy: 9 * nx * ny elements of the storage type, plus nx * ny FP32
 * densities for the local-density encodings or nx * ny bf16 scales for
 * LB_STORE_F16_DEST.  Pure host function. */
size_t lb_state_bytes(const lb_params* p);

/* Create a context and set the state at t = 0 to f_a = [M^-1 m_eq(rho0, u_eq)]_a,
 * the equilibrium of Eq. (3) at every site, taken at u_eq = u0 - F / (2 rho0)
 * with F the Eq. (7) force of the initial density field (FP64).  u0 is thus
 * the Eq. (6) fluid velocity: lb_moments at t = 0 returns (rho0, u0).
 *   workspace        device buffer of at least workspace_bytes (lb_workspace_bytes),
 *                    256-byte aligned, owned by the caller and used by the context
 *                    until lb_destroy.
 *   rho0, ux0, uy0   device FP32 [ny][nx]; ux0/uy0 may be NULL (zero velocity).
 *                    Read during this call only.
 * Validates every rho0 on the device (finite, 0 < rho < 4/b, psi^2 > 0): this
 * call synchronises `stream` once and returns LB_EINVAL if a value is out of
 * range.  On failure *out is set to NULL. */
lb_status lb_init(lb_ctx** out, const lb_params* p, void* workspace, size_t workspace_bytes,
                  const float* rho0, const float* ux0, const float* uy0, void* stream);

/* Advance nsteps >= 0 time steps (asynchronous; captured into graphs of
 * lb_set_launch's chunk size when the stream is not the legacy stream).
 * Instability is detected on the device and reported by lb_check /
 * lb_diagnostics. */
lb_status lb_step(lb_ctx* ctx, int64_t nsteps);

/* Write rho and the half-force velocity v = (sum e f + F/2)/rho (Eq. 6) of the
 * current state into device FP32 [ny][nx] buffers (asynchronous).  Any of the
 * three pointers may be NULL. */
lb_status lb_moments(lb_ctx* ctx, float* rho, float* ux, float* uy);

/* Reductions of the current state over the whole grid and two regions (host
 * pointers).  Synchronises the stream.  Returns LB_EUNSTABLE (and poisons the
 * context) if an instability was flagged; *out is filled in either case. */
lb_status lb_diagnostics(lb_ctx* ctx, const lb_region* in, const lb_region* out, lb_diag* diag);

/* Synchronise the stream and report LB_EUNSTABLE if any step since lb_init
 * flagged an unstable site (the context is then poisoned). */
lb_status lb_check(lb_ctx* ctx);

/* Current time t (host value, no synchronisation). */
int64_t lb_time(const lb_ctx* ctx);

/* Checkpoint: copy the stored state (the post-collision distributions of
 * step t-1, exported as [9][ny][nx] in the storage type, velocity ordering
 * rest, (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1), (-1,-1), (1,-1); for the
 * local-density encodings followed by the [ny][nx] FP32 densities) to / from a
 * device buffer of lb_state_bytes bytes (asynchronous).  lb_set_state also sets
 * the time to t. */
lb_status lb_get_state(lb_ctx* ctx, void* dst);
lb_status lb_set_state(lb_ctx* ctx, const void* src, int64_t t);

/* Launch shape of the step kernel.  strip_rows = rows each wavefront walks;
 * band = strips per tile band (the wavefronts of a workgroup cover `band`
 * strips in y times the rest in x); graph_chunk = steps per captured graph
 * (even, >= 2).  For each: a positive value sets it, 0 keeps the current
 * value, -1 (strip_rows, band only) restores the automatic choice.  Results do
 * not depend on any of them (bitwise). */
lb_status lb_set_launch(lb_ctx* ctx, int32_t strip_rows, int32_t band, int32_t graph_chunk);

/* Release the context and its graphs (not the caller's workspace). */
lb_status lb_destroy(lb_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batched lattices: many independent lattices (each with its own size and
 * parameters, all sharing `store` and `bc`) advanced together.  Every site runs
 * the same arithmetic as lb_step, so each lattice's state is bitwise equal to
 * running it alone.
 * ---------------------------------------------------------------------- */
typedef struct lb_batch lb_batch;

/* Workspace bytes for n lattices with parameter blocks p[0..n-1] (0 if invalid:
 * n < 1, a bad block, differing store/bc, or a store other than LB_STORE_F32 /
 * LB_STORE_F16_LOCAL / LB_STORE_F16_DEST).  Pure host function. */
size_t lb_batch_workspace_bytes(const lb_params* p, int32_t n);

/* Create the batch on a caller-owned device workspace (256-byte aligned, at
 * least lb_batch_workspace_bytes) and set every lattice to its t = 0 state.
 * rho0, ux0, uy0 are host arrays of n device pointers to FP32 [ny_i][nx_i]
 * fields; ux0/uy0 (or entries of them) may be NULL.  The stream must not be the
 * legacy default stream for graph capture (it then launches step by step).
 * Synchronises the stream;
 * LB_EINVAL names the first offending lattice in lb_last_error(). */
lb_status lb_batch_init(lb_batch** out, const lb_params* p, int32_t n, void* workspace,
                        size_t workspace_bytes, const float* const* rho0, const float* const* ux0,
                        const float* const* uy0, void* stream);

/* Advance every lattice by nsteps (asynchronous). */
lb_status lb_batch_step(lb_batch* b, int64_t nsteps);

/* Per-lattice access with the semantics of lb_moments / lb_diagnostics /
 * lb_get_state (lattice index i in the order of lb_batch_init). */
lb_status lb_batch_moments(lb_batch* b, int32_t i, float* rho, float* ux, float* uy);
lb_status lb_batch_diagnostics(lb_batch* b, int32_t i, const lb_region* in, const lb_region* out,
                               lb_diag* diag);
lb_status lb_batch_get_state(lb_batch* b, int32_t i, void* dst);

/* Diagnostics of every lattice in one call (one synchronisation):
 * in[i], out[i] are the regions of lattice i, diag[i] its result (host arrays
 * of n).  Lattices that flagged an unstable site get diag[i].unstable = 1 and
 * keep stepping (their fields are meaningless); the call then returns
 * LB_EUNSTABLE after filling every entry. */
lb_status lb_batch_diagnostics_all(lb_batch* b, const lb_region* in, const lb_region* out, lb_diag* diag);

/* Synchronise; *unstable (may be NULL) receives the number of lattices that
 * flagged an unstable site (LB_EUNSTABLE if any). */
lb_status lb_batch_check(lb_batch* b, int32_t* unstable);

/* Synchronise; seconds[i] (host array of n) = completion time of lattice i in
 * the last lb_batch_step call: from the earliest workgroup start (persistent
 * mode), or the elapsed time of the whole call for every lattice (stepwise). */
lb_status lb_batch_times(lb_batch* b, double* seconds);

/* Launch mode of lb_batch_step:
 *   LB_BATCH_STEPWISE   (default) one launch per time step over the tiles of all
 *                       lattices together (captured in graphs); best throughput;
 *                       lb_batch_times reports the same elapsed time for all.
 *                       Destination-scaled FP16 lattices with an even nx are
 *                       stepped two columns per lane in a second launch.
 *   LB_BATCH_PERSISTENT one launch per lb_batch_step call, one workgroup per
 *                       lattice for all steps; per-lattice completion times.
 * strip_rows: rows per wavefront strip for every lattice, in [1, 64]; 0 = the
 * mode's default (stepwise: a measured height per kernel group, or the heights
 * chosen by lb_batch_tune).  Synchronises the stream.  Results do not depend on
 * either (bitwise). */
enum { LB_BATCH_STEPWISE = 0, LB_BATCH_PERSISTENT = 1 };
lb_status lb_batch_set_launch(lb_batch* b, int32_t mode, int32_t strip_rows);

/* Autotune the strip heights of the stepwise mode on the device at hand.  For each
 * kernel group (one column per lane; two columns per lane, the destination-scaled
 * FP16 lattices with an even nx), the larger first, every height from 1 to 8 is
 * timed over trial_steps launches of the whole batch (1 <= trial_steps <= 1000; the
 * least of three repetitions) and the fastest is kept for the group.  The trial
 * launches read the current state and write only the buffer that the next step
 * overwrites in full, so the state and the time are unchanged; a lattice that is
 * already unstable may set its unstable flag, as its next step would.  Clears a
 * fixed strip height set by lb_batch_set_launch.  rows_out (host array of n, may be
 * NULL) receives each lattice's height.  Stepwise mode only; needs a stream other
 * than the legacy one; synchronises it. */
lb_status lb_batch_tune(lb_batch* b, int32_t trial_steps, int32_t* rows_out);

/* Release the batch and its contexts (not the caller's workspace). */
lb_status lb_batch_destroy(lb_batch* b);

/* Message of the last failure on this thread ("" if none). */
const char* lb_last_error(void);

/* Measurement utility (not part of the method): stream `bytes` (a multiple of
 * 16) from device buffer src to device buffer dst with a plain copy kernel.
 * Used as the attainable-HBM-bandwidth reference next to the step kernel and
 * to calibrate hardware byte counters.  Asynchronous on `stream`. */
lb_status lb_copy_probe(const void* src, void* dst, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LBMP_H */
