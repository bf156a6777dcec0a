/*
 * mmx.h -- C ABI of libmmx, an MI355X (gfx950) implementation of the
 * micromagnetic effective-field + Landau-Lifshitz-Gilbert time step of
 * Claude-SpinDynamics (arxiv 2608.15253).
 *
 * Conventions (all entry points):
 *  - Every call returns mmx_status (0 = MMX_OK, < 0 = error) and never throws.
 *    The message of the last error on the calling thread is mmx_last_error().
 *  - Argument and shape errors are detected before anything is launched.
 *    HIP runtime failures map to MMX_EHIP (message from hipGetErrorString).
 *  - Units are SI: metres, A/m, J/m, J/m^2, J/m^3, tesla, kelvin, seconds.
 *  - Device arrays are owned by the caller (e.g. torch tensors), are not
 *    freed or retained by the library, and must stay alive until the work
 *    queued on the bound stream has finished.  Every device buffer of a
 *    context (twiddle tables, tensor spectrum, stage buffers, controller
 *    state, partial sums) is a region of one workspace of
 *    mmx_workspace_bytes bytes, allocated by mmx_create and freed by
 *    mmx_destroy unless the caller supplies its own with mmx_bind; after
 *    mmx_create no call allocates device memory except mmx_build_demag
 *    (its FP64 tensor staging, freed before it returns) and the network
 *    calls (mmx_fno_*, which own their buffers).
 *  - Magnetisation layout ("D1", Results "A replica-batched engine" and the
 *    replica-batching figure legend: replica-outermost, component-major,
 *    x-fastest): group g, replica r, component c, cell (x, y, z) lives at
 *        m[goff(g) + (r * 3 + c) * N_g + x + n_x * (y + n_y * z)]
 *    with N_g = n_x n_y n_z and goff(g) the sum of 3 R_h N_h over groups h < g.
 *    Element type is float for MMX_F32 contexts and double for MMX_F64.
 *  - All device work is queued asynchronously on the stream given to
 *    mmx_set_stream (default: the null stream).  Calls that return host data
 *    (mmx_rk45 statistics, mmx_build_demag) synchronise that stream.
 *  - Non-finite states: the Heun and rotation correctors (every kernel
 *    variant), the single-cell kernels and the normalised RK4 update raise a
 *    device flag when a new state has a non-finite component.  The
 *    synchronising calls mmx_sync, mmx_rk45 and mmx_relax report it as
 *    MMX_ENONFINITE (and clear it); work already queued is not undone.
 *    mmx_rk45 also returns MMX_ENONFINITE when its step size fell to dt_min
 *    on non-finite error estimates.
 *  - Integrator calls replay captured HIP graphs of their step sequences
 *    (kept between calls with the same arrays and configuration; every setter
 *    call invalidates them), on a library stream ordered after and before the
 *    bound stream by events.
 *  - One context per host thread at a time; calls on one context that overlap
 *    from several threads race.
 */
#ifndef MMX_H
#define MMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mmx_ctx mmx_ctx;

typedef enum { MMX_F32 = 1, MMX_F64 = 2 } mmx_prec;

typedef enum {
  MMX_OK = 0,
  MMX_EINVAL = -1,      /* bad argument value or null pointer                */
  MMX_ESHAPE = -2,      /* grid / group layout not supported or inconsistent */
  MMX_EHIP = -3,        /* HIP runtime error                                 */
  MMX_ESTATE = -4,      /* call out of order (e.g. demag not built)          */
  MMX_EUNSUP = -5,      /* valid but unsupported combination                 */
  MMX_ENONFINITE = -6,  /* a non-finite state was produced on the device     */
  MMX_EDTMIN = -8       /* adaptive step size fell below dt_min              */
} mmx_status;

/* Effective-field terms (Methods, "Physics and discretization"). */
enum {
  MMX_EXCH = 1,            /* six-point Laplacian exchange                     */
  MMX_DMI_INTERFACIAL = 2, /* interfacial DMI; open edges of every term use the
                              free-edge condition of the material's D          */
  MMX_ANIS_UNIAXIAL = 4,   /* uniaxial anisotropy                              */
  MMX_ZEEMAN = 8,          /* applied field                                    */
  MMX_DEMAG = 16,          /* Newell-tensor FFT demagnetisation                */
  MMX_THERMAL = 32,        /* Brown thermal field (Philox4x32-10 noise)        */
  MMX_STT = 64,            /* Slonczewski spin-transfer torque (mmx_set_stt)   */
  MMX_DMI_BULK = 128,      /* bulk DMI (mmx_set_material_ext)                  */
  MMX_ANIS_CUBIC = 256,    /* cubic anisotropy (mmx_set_material_ext)          */
  MMX_RKKY = 512,          /* RKKY interlayer exchange (mmx_set_material_ext)  */
  MMX_ALL_TERMS = 1023
};

/* One geometry advanced for `replicas` independent replicas. */
typedef struct {
  int32_t n[3];          /* cells per axis (x, y, z), each >= 1              */
  double cell[3];        /* cell size per axis, metres                       */
  int32_t pbc[3];        /* 1 = periodic along that axis                     */
  int32_t pbc_images[3]; /* periodic images summed into the demag kernel     */
  int32_t replicas;      /* R >= 1                                           */
} mmx_group;

/* Uniform material of a group (per-cell values: mmx_set_material_cells). */
typedef struct {
  double Ms;     /* saturation magnetisation, A/m (> 0)                     */
  double A;      /* exchange stiffness, J/m                                 */
  double alpha;  /* Gilbert damping                                         */
  double Ku;     /* uniaxial anisotropy constant, J/m^3                     */
  double u[3];   /* anisotropy axis (normalised by the library)             */
  double D;      /* interfacial DMI constant, J/m^2                         */
} mmx_material;

typedef struct {
  double t, dt, err;                    /* time, next step size, last error   */
  int64_t accepted, rejected;           /* step counts                        */
} mmx_rk_stats;

/* Further field terms of a group (Methods, "Physics and discretization":
 * bulk DMI, cubic anisotropy, RKKY interlayer exchange).  SI units. */
typedef struct {
  double Kc1, Kc2;       /* cubic anisotropy constants, J/m^3                 */
  double c1[3], c2[3];   /* cubic axes (c2 made orthogonal to c1; c3 = c1 x c2) */
  double Db;             /* bulk DMI, J/m^2                                   */
  double rkky;           /* RKKY surface energy density sigma, J/m^2          */
  int32_t rkky_z[2];     /* the two coupled cell layers (distinct, < n_z)      */
} mmx_material_ext;

/* Creates a context for `n_groups` geometries.  Checks that device 0 of the
 * current HIP device set is gfx950 and that every axis length can be
 * transformed (FFT sizes with factors 2, 3, 5 only; an even length on
 * periodic x).  Allocates the per-group stage buffers.  *out receives the
 * context; mmx_destroy releases it.  Errors: MMX_EINVAL, MMX_ESHAPE,
 * MMX_EUNSUP, MMX_EHIP. */
mmx_status mmx_create(const mmx_group* groups, int32_t n_groups, mmx_prec prec,
                      mmx_ctx** out);
void mmx_destroy(mmx_ctx* ctx);

/* Binds the HIP stream (hipStream_t passed as void*) used by every later call. */
mmx_status mmx_set_stream(mmx_ctx* ctx, void* hip_stream);

/* Size in bytes of the context's device workspace (all of its device
 * buffers; Methods, "GPU implementation": state and stage buffers stay on the
 * device, with no per-step transfer). */
mmx_status mmx_workspace_bytes(const mmx_ctx* ctx, size_t* bytes);

/* Moves the context's workspace into caller-owned device memory `ws` (at
 * least mmx_workspace_bytes bytes, 256-byte aligned, e.g. a torch tensor;
 * the caller keeps it alive until mmx_destroy or the next mmx_bind) and binds
 * `hip_stream` like mmx_set_stream.  Synchronises the previous stream, copies
 * the current contents (tensor spectrum, tables, parameters) and frees the
 * library's own allocation; captured graphs are dropped.  ws = null moves the
 * workspace back into a library allocation.  MMX_EINVAL for a short or
 * misaligned workspace. */
mmx_status mmx_bind(mmx_ctx* ctx, void* ws, size_t bytes, void* hip_stream);

/* Material of group g (Methods, "Physics and discretization"). */
mmx_status mmx_set_material(mmx_ctx* ctx, int32_t group, const mmx_material* mat);

/* Field-term mask (bitwise or of the MMX_* term flags) used by every
 * evaluation; default MMX_EXCH|MMX_DMI_INTERFACIAL|MMX_ANIS_UNIAXIAL|
 * MMX_ZEEMAN|MMX_DEMAG. */
mmx_status mmx_set_terms(mmx_ctx* ctx, uint32_t mask);

/* Applied flux density B (tesla, host array of 3) of group g; H = B / mu0. */
mmx_status mmx_set_field(mmx_ctx* ctx, int32_t group, const double B_tesla[3]);

/* Temperature (K) and 64-bit Philox key of every replica of group g (host
 * arrays of length R_g).  Brown field sigma = sqrt(2 alpha kB T /
 * (mu0^2 Ms V gamma0 dt)) (Results, "A replica-batched engine"); noise
 * eta ~ N(0,1) from Philox4x32-10 (Salmon et al. 2011) with key = seed and
 * counter = (cell, step low word, step high word, 0), Box-Muller on the four
 * uniforms (x + 1/2) 2^-32, first three normals used as (x, y, z). */
mmx_status mmx_set_thermal(mmx_ctx* ctx, int32_t group, const double* T_per_replica,
                           const uint64_t* seed_per_replica);

/* Builds the demag kernel of every group in FP64 on the device: Newell tensor
 * (Newell, Williams & Dunlop 1993) per offset, closed form at scaled
 * Chebyshev distance <= 2 and Gauss-Legendre dipole quadrature beyond,
 * periodic images summed on periodic axes, zero at the padded Nyquist offset,
 * FFT, scaled by -Ms / (Px Py Pz), reduced to the real, parity-compressed
 * (Px/2+1)(Py/2+1)(Pz/2+1) block per component and rounded to the context
 * precision.  Requires the material to be set.  Synchronous. */
mmx_status mmx_build_demag(mmx_ctx* ctx);

/* Further field terms of group `group` (enabled by MMX_DMI_BULK,
 * MMX_ANIS_CUBIC, MMX_RKKY in the term mask):
 *   bulk DMI: energy density Db m.(curl m), H = -(2 Db / mu0 Ms) curl m with
 *     central differences; open edges add (Db/2A) e_a x m to the free-edge
 *     derivative of the shared exchange/DMI ghosts on every axis (from the
 *     material's Db, whatever the mask);
 *   cubic anisotropy: energy density Kc1 (m1^2 m2^2 + m2^2 m3^2 + m3^2 m1^2)
 *     + Kc2 m1^2 m2^2 m3^2, m_i = m.c_i, H = -(1/mu0 Ms) dE/dm;
 *   RKKY: surface energy density -sigma m(z0).m(z1) between cell layers
 *     z0 = rkky_z[0], z1 = rkky_z[1]: H = sigma / (mu0 Ms dz) m(other layer).
 * mmx_energy reports bulk DMI in the DMI slot, cubic anisotropy in the
 * anisotropy slot (from its energy density) and RKKY in the exchange slot.
 * These terms run on the field kernels of the staged path (the register row
 * kernels and the replica-resident path do not take them).  MMX_EINVAL for a
 * null pointer, Db != 0 with A = 0, zero or parallel cubic axes, or RKKY
 * layers that are equal or out of range. */
mmx_status mmx_set_material_ext(mmx_ctx* ctx, int32_t group, const mmx_material_ext* ext);

/* Per-cell exchange stiffness of group `group` (Methods, per-cell materials):
 * A (host double[N], J/m, x-fastest like one component of m; copied) replaces
 * the material's A in the exchange term, with the pair coupling given by the
 * harmonic mean 2 A_i A_j / (A_i + A_j) (0 if both vanish), H_i = (2 / mu0 Ms)
 * sum_j A_ij (m_j - m_i) / d^2, a ghost neighbour taking A_i; the edge
 * conditions use D / 2A_i and Db / 2A_i (0 where A_i = 0).  A = null goes
 * back to the uniform A.  Field kernels of the staged path only (like
 * mmx_set_material_ext).  Synchronous.  MMX_EINVAL for a negative or
 * non-finite value. */
mmx_status mmx_set_exchange_cells(mmx_ctx* ctx, int32_t group, const double* A);

/* Per-cell materials of group `group` (Methods, "Physics and
 * discretization": material parameters per cell).  Ms, A, alpha, Ku, D:
 * device arrays of N_g values each (x fastest, like one component of m),
 * element type of the context, copied (the caller may free them on return);
 * a null pointer leaves that parameter uniform (the group's material; for A
 * this also drops an earlier mmx_set_exchange_cells).  Fields: every term
 * with a 1 / (mu0 Ms) prefactor takes the cell's Ms_i; the demag convolution
 * acts on M_j = Ms_j m_j; anisotropy 2 Ku_i / (mu0 Ms_i) (m.u) u; the
 * interfacial DMI keeps each cell's energy density D_i [m_z div m - (m.grad)
 * m_z], so a neighbour pair couples with (D_i + D_j) / 2 and the field of
 * cell i along x is (1 / mu0 Ms_i dx) [D_{i,i+1} m_z(i+1) - D_{i-1,i}
 * m_z(i-1)] (similarly y, and the matching terms of H_z); a ghost neighbour
 * takes the edge cell's D_i, the edge condition D_i / 2A_i; exchange as in
 * mmx_set_exchange_cells with 1 / (mu0 Ms_i); the torque and the Brown field
 * use alpha_i and Ms_i; the spin-transfer b_J uses Ms_i; energies weigh each
 * cell by its Ms_i.  The group's material must be set first (its Ms is the
 * reference of the derived arrays).  These parameters run on the field
 * kernels of the staged path (the register row kernels, the
 * replica-resident and the single-cell paths do not take them; the learned
 * demag stages reject them).  Synchronous.  MMX_EINVAL for Ms <= 0, A < 0,
 * alpha < 0 or a non-finite value, MMX_ESTATE before mmx_set_material. */
mmx_status mmx_set_material_cells(mmx_ctx* ctx, int32_t group, const void* Ms, const void* A,
                                  const void* alpha, const void* Ku, const void* D);

/* Slonczewski spin-transfer torque of group `group` (Methods, "Physics and
 * discretization": spin torques added per integrator stage; Results, the
 * replica-batched STT switching sweep with a current density per replica).
 * J: host double[R] current densities (A/m^2), copied; p: fixed-layer
 * direction (normalised here); P: polarisation; Lambda > 0: asymmetry;
 * eps_prime: field-like coefficient.  With MMX_STT in the term mask every
 * torque evaluation (mmx_torque, all integrators) adds, in the
 * Landau-Lifshitz form of the LLG equation,
 *   gamma' mu0 b_J [(eps - alpha eps') m x (m x p) - (eps' + alpha eps) m x p],
 *   b_J = hbar J / (mu0 e Ms d), eps = P Lambda^2 / ((Lambda^2 + 1) +
 *   (Lambda^2 - 1) m.p), d = the group's thickness n_z cell_z,
 * i.e. the Gilbert-form torque gamma0 mu0 b_J [eps m x (m x p) - eps' m x p]:
 * J > 0 drives m away from p.  It does not enter mmx_field or mmx_energy.
 * Runs on the staged path (mmx_heun returns MMX_EUNSUP under
 * MMX_PATH_FUSED).  Synchronous.  MMX_EINVAL for null pointers, p = 0,
 * Lambda <= 0 or non-finite values. */
mmx_status mmx_set_stt(mmx_ctx* ctx, int32_t group, const double* J, const double p[3],
                       double P, double Lambda, double eps_prime);

/* Effective field H (A/m, device, layout D1) at state m (device, D1) for
 * all groups, with the enabled terms; the thermal term uses `step` and `dt`.
 * Methods, "Physics and discretization". */
mmx_status mmx_field(mmx_ctx* ctx, const void* m, void* H, uint64_t step, double dt);

/* LLG right-hand side dm/dt (1/s, device, D1) at m (LLG equation, Methods):
 * -gamma' mu0 [m x H + alpha m x (m x H)], gamma' = gamma0 / (1 + alpha^2). */
mmx_status mmx_torque(mmx_ctx* ctx, const void* m, void* dmdt, uint64_t step, double dt);

/* n_steps Stratonovich Heun steps of size dt, in place on m (device, D1),
 * steps numbered step0 .. step0+n_steps-1 for the thermal noise, which is
 * drawn once per step and shared by predictor and corrector (Methods,
 * "Replica batching"; Results, finite-temperature comparison).  The corrector
 * is normalised.  If t_switch (device double[R_total]) is not null, entries
 * still negative receive (step+1)*dt at the first step after which the
 * replica's mean m_z is negative. */
mmx_status mmx_heun(mmx_ctx* ctx, void* m, double dt, int64_t n_steps, uint64_t step0,
                    void* t_switch);

/* n_steps steps of the norm-exact Depondt-Mertens rotation scheme (Results,
 * "A replica-batched engine": Rodrigues update, |m| = 1 to round-off;
 * Methods, "Integrators" and "Replica batching"), in place on m (device, D1).
 * The LLG equation is taken as dm/dt = Omega x m, Omega = gamma' mu0 (H +
 * alpha m x H).  Per step, with the thermal field drawn once (as mmx_heun):
 * Omega_1 at m; predictor m~ = rotation of m about Omega_1 by |Omega_1| dt;
 * Omega_2 at m~; the new state is the rotation of m about (Omega_1 +
 * Omega_2)/2 by |Omega_1 + Omega_2| dt/2.  FP64 runs take no normalisation;
 * FP32 runs renormalise the new state (the rounding of cos|w| near 1 would
 * otherwise repeat step after step when the rotation barely changes).  Step
 * numbering and t_switch as in mmx_heun.  Runs on the staged path
 * (MMX_EUNSUP under MMX_PATH_FUSED). */
mmx_status mmx_depondt(mmx_ctx* ctx, void* m, double dt, int64_t n_steps, uint64_t step0,
                       void* t_switch);

/* Retire/refill trials of the rotation scheme (Results, "A replica-batched
 * engine": a trial that meets its stop condition is frozen and its slot
 * restarts with a fresh noise stream).  Every replica r starts trial g = 0
 * from m (device, D1) at step step0; after each step, a replica whose mean
 * m_z is negative ends its trial: the trial's length (steps since its start
 * + 1) * dt goes to times[r * cap + g] (device double[R_total][cap], entries
 * set to -1 first, only the first cap trials recorded), counts[r] (device
 * int32[R_total], set to 0 first) is incremented, and the replica restarts
 * at the next step from its row of m_init (device, D1, not modified) with
 * trial g + 1, whose thermal noise uses counter word 3 = g + 1 and step
 * numbers counted from the trial's start (trial 0 is the noise of
 * mmx_depondt).  Each call starts a fresh set of trials.  Single-cell groups
 * without demag keep the bookkeeping in the replica's thread (as mmx_depondt
 * does under MMX_PATH_AUTO).  MMX_EINVAL for null m, m_init or counts,
 * cap < 0, or null times with cap > 0. */
mmx_status mmx_depondt_refill(mmx_ctx* ctx, void* m, const void* m_init, double dt,
                              int64_t n_steps, uint64_t step0, void* times, int32_t cap,
                              void* counts);

/* n_steps classical fourth-order Runge-Kutta steps of fixed size dt
 * (Methods, "Integrators": RK4, four field evaluations per step), in place
 * on m (device, D1): k1 = f(m), k2 = f(m + dt/2 k1), k3 = f(m + dt/2 k2),
 * k4 = f(m + dt k3), m <- normalise(m + dt (k1/6 + k2/3 + k3/3 + k4/6)); the
 * stage states are not normalised.  Thermal terms are rejected
 * (MMX_EUNSUP). */
mmx_status mmx_rk4(mmx_ctx* ctx, void* m, double dt, int64_t n_steps);

/* on = 0: damping-only dynamics (the relaxation dynamics of the Methods'
 * damping-only relaxer): every torque evaluation of mmx_torque, mmx_rk45 and
 * mmx_rk4 drops the precession term, dm/dt = -gamma' mu0 alpha m x (m x H)
 * (gamma' unchanged); mmx_heun and mmx_depondt* return MMX_EUNSUP.  on = 1
 * (default): the full LLG equation. */
mmx_status mmx_set_precession(mmx_ctx* ctx, int32_t on);

/* Damping-only relaxation (Methods, "Integrators": damping-only relax) of m
 * (device, D1, in place): mmx_rk45 on the damping-only dynamics with
 * tolerance tol, in chunks of 10 ps of simulated time (each chunk starts from
 * the controller's last proposal before it was clipped to the chunk's end,
 * the first with 1e-14 s), until the max over all replicas and cells of
 * |dm/dt| is <= torque_tol (1/s) or the time reaches t_max.  stats (host,
 * nullable): final time, last proposal, last error, summed step counts;
 * max_torque (host, nullable): the final max |dm/dt|.  Synchronous; thermal
 * terms are rejected (MMX_EUNSUP); MMX_EINVAL for torque_tol < 0, t_max <= 0
 * or tol <= 0. */
mmx_status mmx_relax(mmx_ctx* ctx, void* m, double torque_tol, double t_max, double tol,
                     mmx_rk_stats* stats, double* max_torque);

/* Adaptive Dormand-Prince 5(4) relaxation (Methods, "Integrators") of m
 * (device, D1, in place) from t0 to t_end with absolute tolerance tol on the
 * max-over-cells Euclidean norm of the embedded error; first attempt dt0;
 * dt <- dt clamp(0.9 (tol/err)^(1/5), 0.2, 5), limited to 1e-11 s and to the
 * time left; the candidate is normalised before the first-same-as-last stage.
 * Step control runs on the device.  If dt_replay (host, n_replay entries) is
 * not null the given step sizes are taken in order without control.  If
 * energy_trace (device double, trace_cap entries) is not null the total
 * energy after each accepted step is appended (entry 0 = initial state).
 * Thermal terms are rejected (MMX_EUNSUP).  stats (host) receives the final
 * controller state.  Synchronous.  MMX_EDTMIN if dt falls below 1e-20 s. */
mmx_status mmx_rk45(mmx_ctx* ctx, void* m, double t0, double t_end, double tol, double dt0,
                    const double* dt_replay, int64_t n_replay, void* energy_trace,
                    int64_t trace_cap, mmx_rk_stats* stats);

/* Synchronises the bound stream; MMX_ENONFINITE if a corrector or a
 * normalised update produced a non-finite state since the last check (the
 * flag is cleared), else MMX_OK. */
mmx_status mmx_sync(mmx_ctx* ctx);

/* Checkpoint of an adaptive run (Methods, "Integrators"): after mmx_rk45 or
 * mmx_rk45_resume (not a dt replay), the controller state (time, the last
 * step-size proposal before clipping to t_end, last error, step counts) and
 * the first-same-as-last slope k1 of every replica (device values of the
 * final state), as a host blob: header, then k1 in layout D1 with the
 * context's element type.  blob = null: *bytes receives the size.  The
 * magnetisation itself is the caller's array and is not included.
 * Synchronous.  MMX_ESTATE if no adaptive run precedes it, or another
 * integrator or a setter was called since (they reuse the stage buffers or
 * change the dynamics). */
mmx_status mmx_checkpoint(const mmx_ctx* ctx, void* host_blob, size_t* bytes);

/* Loads a checkpoint into a context of the same precision and groups (same
 * mmx_group descriptions; materials, field and terms must be set as when it
 * was taken); the next mmx_rk45_resume continues from it.  Synchronous.
 * MMX_EINVAL for a blob that is not a checkpoint or too short, MMX_ESHAPE
 * for another layout. */
mmx_status mmx_restore(mmx_ctx* ctx, const void* host_blob, size_t bytes);

/* Continues the adaptive run of the last mmx_rk45 / mmx_rk45_resume call or
 * of the restored checkpoint from its time and step-size proposal to t_end,
 * with the saved first-same-as-last slope as the first stage (m must be the
 * state the run ended in); arguments, output and errors as mmx_rk45.  A run
 * continued in a context restored from a checkpoint equals its continuation
 * in the original context bit for bit. */
mmx_status mmx_rk45_resume(mmx_ctx* ctx, void* m, double t_end, double tol, void* energy_trace,
                           int64_t trace_cap, mmx_rk_stats* stats);

/* Accepted step sizes of the last mmx_rk45 call (host array, up to cap
 * entries); *count receives the number available. */
mmx_status mmx_rk45_dts(mmx_ctx* ctx, double* dts, int64_t cap, int64_t* count);

/* Energy per term (J) of every replica: E (device double[R_total][6]) in the
 * order exchange, DMI, demag, anisotropy, Zeeman, total;
 * E = V sum_i [-(mu0 Ms / 2) m.(H_ex + H_dmi + H_d + H_anis) - mu0 Ms m.H_Z]. */
mmx_status mmx_energy(mmx_ctx* ctx, const void* m, void* E);

/* Topological charge of layer z = 0 of every replica, Q (device
 * double[R_total]) = (1/4 pi) sum m.(d_x m x d_y m) dx dy with central
 * differences (periodic wrap, the cell itself beyond open edges). */
mmx_status mmx_topological_charge(mmx_ctx* ctx, const void* m, void* Q);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the charges of
 * mmx_topological_charge, equal to them bit for bit, computed with the
 * per-workgroup partial sums in a static device array of the library (1 MiB
 * per device, 131072 doubles, reserved when the library is loaded and set up
 * by mmx_create, held until the process ends) instead of a buffer allocated
 * per call.  Allocates nothing and does not synchronise: the result is
 * queued on the bound stream.  The array is shared by every context on a
 * device, so calls on one device that overlap (several streams or host
 * threads) race; calls queued on one stream are ordered.  MMX_EINVAL if a
 * group needs more partial sums (replicas x min(256, ceil(n_x n_y / 256)))
 * than the array holds, before anything is launched. */
mmx_status mmx_topological_charge_noalloc(mmx_ctx* ctx, const void* m, void* Q);

/* Tile sizes of group g: tiles[0] = grid rows per workgroup of the x
 * transform / local-field kernels, tiles[1] = spectrum columns per workgroup
 * of the y transform, tiles[2] = of the z transform, or, for 3-D groups of
 * at most 8 layers, of the fused y-z pass (which then takes no y tile).
 * Results are identical for every valid choice; only speed changes.
 * mmx_set_tiles rejects sizes outside [1, n_y] / [1, n_x/2 + 1] or beyond the
 * LDS of a workgroup (64 KiB; the fused y-z pass: the device's maximum)
 * (MMX_EINVAL) and synchronises the stream.  mmx_autotune times one field
 * evaluation of every group (after mmx_build_demag) for candidate sizes
 * 1, 2, 4, ..., 32 per tile, keeps the fastest, and synchronises; it
 * overwrites the library's stage buffers, not caller arrays. */
/* Execution path of mmx_heun.  MMX_PATH_STAGED: every field evaluation is
 * three (2-D and few-layer 3-D) or five (other 3-D) launches over all
 * replicas, with the spectrum in
 * HBM.  MMX_PATH_FUSED: one workgroup per replica runs whole Heun steps with
 * the replica's half spectrum resident in LDS (2-D films whose spectrum, row
 * and column scratch fit the device's LDS per workgroup; mmx_heun returns
 * MMX_EUNSUP otherwise).  MMX_PATH_AUTO (default): fused where it fits, staged
 * elsewhere.  Both paths compute the same arithmetic per transform line and
 * per cell.  Under AUTO and FUSED, single-cell groups without the demag term
 * (macrospins) advance every replica for all steps in one thread's registers
 * (mmx_heun and mmx_depondt; results equal the staged path to round-off). */
enum { MMX_PATH_AUTO = 0, MMX_PATH_STAGED = 1, MMX_PATH_FUSED = 2 };
mmx_status mmx_set_path(mmx_ctx* ctx, int32_t path);

mmx_status mmx_set_tiles(mmx_ctx* ctx, int32_t group, const int32_t tiles[3]);
mmx_status mmx_get_tiles(mmx_ctx* ctx, int32_t group, int32_t tiles[3]);
mmx_status mmx_autotune(mmx_ctx* ctx);

/* ------------------------------------------------------------------------
 * Learned demag surrogate: a Fourier neural operator h = f(m) ~ H_demag / Ms
 * for films of H x W cells (an extension; not in the paper).
 * Network: features [m, x/W - 1/2, y/H - 1/2] -> 1x1 lift to C channels ->
 * L layers of [truncated DFT (kx < M1, ky in [0, M2) u [H - M2, H)) ->
 * per-mode complex C x C mixing -> inverse real DFT, plus a 1x1 map and
 * bias, GELU except after the last layer] -> 1x1 to Cp -> GELU -> 1x1 to 3.
 * The 1x1 maps run as BF16 matrix-core GEMMs with FP32 accumulation
 * (use_mfma = 1) or in FP32 (use_mfma = 0); transforms, mixing and reductions
 * are FP32.  All arrays are FP32 device pointers owned by the caller:
 * m, h, target [B][3][H][W] (x fastest); params and grads packed as
 *   P[C][5], p[C], then per layer R[M1][2 M2][C][C] (complex, re/im
 *   interleaved), W[C][C], b[C], then Q1[Cp][C], q1[Cp], Q2[3][Cp], q2[3],
 * mmx_fno_param_count floats in total; moments (Adam) 2x that.
 * The loss is the batch mean of |h - t|^2 / |t|^2 per sample.
 * mmx_fno_backward differentiates the last mmx_fno_forward (its activations
 * stay in library buffers) and overwrites grads.  Errors: MMX_EINVAL for bad
 * sizes / nulls, MMX_EUNSUP beyond C, Cp <= 128, batch <= 64, MMX_ESTATE for a
 * backward without forward.  mmx_fno_create allocates every device buffer
 * the forward and backward passes use (sized for batch_max); forward,
 * backward and Adam allocate nothing.  Work is queued on the FNO's stream;
 * the loss is returned synchronously when `loss` is not null.
 * ------------------------------------------------------------------------ */
typedef struct mmx_fno mmx_fno;
mmx_status mmx_fno_create(int32_t H, int32_t W, int32_t C, int32_t M1, int32_t M2, int32_t L,
                          int32_t Cp, int32_t batch_max, int32_t use_mfma, mmx_fno** out);
void mmx_fno_destroy(mmx_fno* f);
mmx_status mmx_fno_set_stream(mmx_fno* f, void* hip_stream);
mmx_status mmx_fno_param_count(const mmx_fno* f, int64_t* n);
/* Seeded initial weights (scaled normals; spectral weights uniform in [0, 1/C^2)). */
mmx_status mmx_fno_init(mmx_fno* f, float* params, uint64_t seed);
mmx_status mmx_fno_forward(mmx_fno* f, const float* params, const float* m, float* h,
                           int32_t batch);
mmx_status mmx_fno_backward(mmx_fno* f, const float* params, const float* h, const float* target,
                            float* grads, double* loss);
/* Adam (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8) on every float of
 * params; moments = [first moments | second moments], zero before step t = 1. */
mmx_status mmx_fno_adam(mmx_fno* f, float* params, const float* grads, float* moments, double lr,
                        int64_t t);

/* ---- RK45 with learned demag stages --------------------------------------
 * The adaptive Dormand-Prince integration of mmx_rk45 (Methods,
 * "Integrators"; same tableau, controller, dt_max and dt_min) in which stages
 * 2-6 of an attempt take the demagnetising field from the network `net` with
 * parameters `params` (device, FP32, layout above) instead of the FFT
 * convolution: Hd = Ms * f(m) + (0, 0, -Ms m_z if residual_mz).  Stage 7, at
 * the candidate point, and the first stage of the run use the exact field.
 * (The learned stages and their gate are an extension, not a method of the
 * paper.)  Gate: when the controller accepts such an attempt, the network is evaluated
 * at the candidate state m7 and compared with the exact stage-7 field; the
 * step is kept iff, for every replica, |Hd_net - Hd_exact|_2 / |Hd_exact|_2
 * <= gate_tol over the film.  Otherwise the attempt (and equally an attempt
 * the controller rejects) is discarded and repeated from the same state and
 * step size with the exact field in every stage; after a gate failure the
 * next exact_after_fail accepted steps are also exact.  With gate_tol = 0 (or
 * unusable weights) every kept step is an exact one and the result equals
 * mmx_rk45's bit for bit.  Requires: FP32 context, one group, a film
 * (nz = 1) of net's H x W grid (ny = H, nx = W), replicas <= net's
 * batch_max, demag term on and built, no thermal term.  The run is driven
 * from the host (one synchronisation per attempt, one per gate check) on the
 * context's stream; net's own stream is left unchanged.  gate_log (host,
 * optional, gate_cap entries) receives the largest replica error of each
 * gate check in order; stats (host, optional) the counters below.
 * Errors: EINVAL, ESHAPE, ESTATE, EUNSUP, EHIP, EDTMIN as for mmx_rk45. */
typedef struct {
  double t, dt, err;            /* final time, next step size, last error estimate */
  int64_t accepted, rejected;   /* accepted steps; controller rejections of exact attempts */
  int64_t surrogate_steps;      /* accepted steps whose stages 2-6 used the network */
  int64_t exact_steps;          /* accepted steps with the exact field in every stage */
  int64_t gate_checks, gate_failures;
  int64_t surrogate_rejected;   /* network attempts rejected by the controller (repeated) */
  double gate_max_passed;       /* largest gate error among the kept steps */
} mmx_surrogate_stats;
mmx_status mmx_rk45_surrogate(mmx_ctx* ctx, mmx_fno* net, const float* params, void* m, double t0,
                              double t_end, double tol, double dt0, double gate_tol,
                              int32_t residual_mz, int32_t exact_after_fail, double* gate_log,
                              int64_t gate_cap, mmx_surrogate_stats* stats);

/* Measurement support (not part of the method).  mmx_profile_enable(ctx, 1)
 * clears the statistics and brackets every later kernel launch of ctx with a
 * pair of HIP events on the bound stream; mmx_profile_enable(ctx, 0) stops.
 * mmx_profile_get reports, for kernel index idx (0 <= idx < *n_kernels), its
 * name (NUL-terminated, truncated to name_cap), the summed event time in ms
 * and the launch count; with idx < 0 only *n_kernels is written.  Both calls
 * synchronise the stream. */
mmx_status mmx_profile_enable(mmx_ctx* ctx, int32_t on);
mmx_status mmx_profile_get(mmx_ctx* ctx, int32_t idx, char* name, int32_t name_cap,
                           double* total_ms, int64_t* count, int32_t* n_kernels);

const char* mmx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MMX_H */
