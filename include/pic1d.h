/*
 * pic1d.h -- C ABI of the MI355X (gfx950) library for the 1D particle-in-cell
 * hot path of RICS-driven pair cascades on dipole field lines.
 *
 * What is computed (paper: Mahlmann, Philippov, Soudais, Beloborodov and
 * Sironi, "1D PIC Simulations of Resonant Scattering-Driven Pair Cascades in
 * Magnetar Magnetospheres"):
 *   - field-line geometry B(s), mu(s), r(s) of a dipole line (Appendix B.2);
 *   - per step, for every particle: field gather, the RICS drag force by
 *     Strang splitting with the drag limiter, implicit midpoint and damping
 *     branches (Sec. 3, Eq. implicit), or a stochastic scattering event with
 *     probability Ndot dt (Sec. 3) and recoil (Appendix A), the Lorentz push,
 *     the move, a charge-conserving current deposit, absorption at the
 *     conducting stellar surface (Sec. 3);
 *   - conversion of photons with E >= 2 m_e c^2 into e-/e+ pairs, limited by
 *     n_max (Sec. 3), and refill of the surface atmosphere (Appendix B.1);
 *   - Ampere's law with the static twist current, dE/dt = 4 pi (j_ext - j) (Sec. 3).
 *
 * Code units: one cell, one step; c = cfl cells/step; n0 = ppc0 macro-particles
 * per cell per species; skin depth d0_cells at n0.  Positions are an int32 cell
 * index plus a float32 offset in [0,1); momenta u = gamma*beta are float32; the
 * field E and the diagnostics are float64.
 *
 * Conventions common to all calls:
 *   - Every function returns a pic1d_status (0 = PIC1D_OK) unless noted.
 *   - Pointers documented as "host" point to caller-owned host memory that is
 *     read or written during the call only.  Pointers documented as "device"
 *     point to device memory of the current HIP device (e.g. torch tensors).
 *   - All device work is enqueued on the hipStream_t given in the config;
 *     calls that return data to host buffers synchronise that stream.
 *   - One state handle must not be used from two threads at once.
 *   - After PIC1D_ECAPACITY or PIC1D_ENONFINITE the state is frozen: further
 *     pic1d_step calls return PIC1D_ESTATE; moments and particles stay readable
 *     but reflect the partially completed step in which the error occurred.
 */
#ifndef PIC1D_H
#define PIC1D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PIC1D_OK = 0,
    PIC1D_EINVAL = -1,      /* invalid argument or config                      */
    PIC1D_ENOMEM = -2,      /* workspace too small                             */
    PIC1D_ECAPACITY = -3,   /* a species of a line ran out of particle slots   */
    PIC1D_EDEVICE = -4,     /* a HIP runtime call failed                       */
    PIC1D_ENONFINITE = -5,  /* a momentum or field value became NaN/Inf        */
    PIC1D_ESTATE = -6       /* state frozen by an earlier error                */
} pic1d_status;

/* RICS backends: how F_hat, Ndot_hat are evaluated (photon energy is always
 * the closed form of Appendix A.3, Eq. perpemit). */
enum { PIC1D_RICS_OFF = 0,     /* no radiation reaction                          */
       PIC1D_RICS_EXACT = 1,   /* closed forms of Eqs. scatteringNdot, contdrag  */
       PIC1D_RICS_TABLE = 2,   /* bilinear (log10 gamma, s) table of the same    */
       PIC1D_RICS_MLP = 3 };   /* the trained surrogate network (pic1d_mlp_*)    */

/* The thermal photon field RICS scatters (Sec. 2.2 and Sec. 5). */
enum { PIC1D_FIELD_RADIAL = 0,     /* photons stream radially from the star, pi/x^2 sr
                                      (Sec. 2.2: the radial beam behind Eq. contdrag) */
       PIC1D_FIELD_DISK = 1 };     /* the finite stellar disk (Sec. 5): the rate and
                                      force integrated over the cone of half-angle
                                      asin(1/x) filled by the star, at uniform
                                      intensity, by a 24 x 24 Gauss-Legendre product
                                      rule in (cos t, phi); TABLE backend only, the
                                      table built on the device in float64        */

/* Where a photon with E >= 2 m_e c^2 converts. */
enum { PIC1D_CONV_IMMEDIATE = 0,   /* at the emission point (Sec. 3)              */
       PIC1D_CONV_CURVATURE = 1 }; /* where its angle to the curved line reaches
                                      arcsin(2 m_e c^2 / E): s' = s +- R_curv asin */

/* Direction of the de-excitation photon in the rest frame of the excited lepton
 * (Appendix A.2-A.3).  The lab photon energy and the recoil follow from the
 * rest-frame energy E_gamma(theta) of Appendix A.2, the lepton recoiling along B,
 * boosted back with gamma_e = gamma (1+2b)^-1/2 (Eq. scatlim1; no boost where
 * gamma_e < 1); the cosine from the lepton's motion is drawn from the second word of
 * the event's Philox block.  The paper defers the pattern to an external reference:
 * the non-perpendicular patterns are readings. */
enum { PIC1D_EMIT_PERPENDICULAR = 0, /* cosine 0: eps = gamma (1 - (1+2b)^-1/2) (Eq.
                                        perpemit), the lepton keeps gamma_e       */
       PIC1D_EMIT_ISOTROPIC = 1,     /* cosine uniform on [-1, 1]                   */
       PIC1D_EMIT_DIPOLE = 2 };      /* density 3/8 (1 + cosine^2), the classical
                                        cyclotron pattern summed over polarisations */

/* Initial pair plasma of a line (Sec. 3: homogeneous e-/e+ plasma). */
enum { PIC1D_INIT_COLD = 0,    /* u = 0                                          */
       PIC1D_INIT_HOT = 1,     /* gamma log-uniform in [1, init_gamma_max], random sign */
       PIC1D_INIT_STREAM = 2,  /* e+ at +gamma*init_beta, e- opposite (along j)  */
       PIC1D_INIT_EMPTY = 3 }; /* no particles                                   */

/* Species index. */
enum { PIC1D_E_PAIR = 0, PIC1D_P_PAIR = 1, PIC1D_E_ATM = 2, PIC1D_ION = 3, PIC1D_NSPECIES = 4 };

/* Moment flags. */
enum { PIC1D_MOM_INSTANT = 0, PIC1D_MOM_AVERAGE = 1, PIC1D_MOM_RESET = 2 };

/* Counter slots of pic1d_moments.counters. */
enum { PIC1D_CNT_EVENTS = 0,          /* stochastic RICS events                 */
       PIC1D_CNT_PAIRS = 1,           /* e-/e+ pairs created                    */
       PIC1D_CNT_ESCAPED = 2,         /* photons that did not convert           */
       PIC1D_CNT_ABSORBED = 3,        /* particles absorbed by the walls        */
       PIC1D_CNT_PSC_CLIPPED = 4,     /* event probabilities Ndot*dt clipped at 1 */
       PIC1D_CNT_LIMITED = 5,         /* drag half steps taken by the damping branch */
       PIC1D_CNT_NEWTON = 6,          /* drag half steps that needed Newton iterations */
       PIC1D_CNT_ATM = 7,             /* atmosphere (e-, ion) pairs injected    */
       PIC1D_CNT_PUSHED = 8,          /* particle-steps pushed                  */
       PIC1D_CNT_DRAWS = 9,           /* Philox draws of event decisions        */
       PIC1D_CNT_MLP_EVALS = 10,      /* surrogate-network evaluations executed (one per lane
                                         and wavefront-wide call, idle lanes included) */
       PIC1D_CNT_ANNIHILATED = 11,    /* e-/e+ pairs annihilated at the density limit */
       PIC1D_CNT_PUSHED_IONS = 12,    /* ion steps among PIC1D_CNT_PUSHED               */
       PIC1D_CNT_MLP_NEEDED = 13,     /* surrogate evaluations the step needs: 2 per lepton
                                         step in the continuous regime plus its refinements,
                                         1 in the stochastic regime                     */
       PIC1D_NCOUNTERS = 16 };

typedef struct {
    double r_eq;              /* equatorial radius of the line, R_max / R*   */
    int32_t n_cells;          /* cells, uniform in arc length, 2..2^26; at   */
                              /*   most 2^27 cells over all lines            */
    int32_t ppc_init;         /* initial e-/e+ pairs per cell (>= 0)         */
    int32_t init_mode;        /* PIC1D_INIT_*                                */
    int32_t pad0;
    double init_gamma_max;    /* HOT: upper end of the gamma range           */
    double init_beta;         /* STREAM: |beta| of both species (< 1)        */
    int64_t capacity[4];      /* particle slots per species; 0 = default     */
} pic1d_line;

typedef struct {
    int32_t n_lines;          /* >= 1 field lines, advanced together         */
    int32_t emission;         /* PIC1D_EMIT_*: rest-frame photon direction    */
    const pic1d_line* lines;  /* host, n_lines entries                       */
    double b_pole;            /* B_star / B_QED at the pole surface (10)     */
    double cfl;               /* c0/c (0.5), cells per step at c             */
    double d0_cells;          /* cells per skin depth at n0 (48)             */
    double ppc0;              /* macro-particles per cell per species at n0  */
    double j_twist;           /* j_psi / (n0 e c), signed along +s           */
    double kT_keV;            /* photon temperature                          */
    double eta_min;           /* eta_min prefactor: tau_min w_p0 = eta_min (n_psi/n0)^(1/2) */
    double b_thr;             /* stochastic regime where b >= b_thr (0.1)    */
    double mass_ratio;        /* m_i / m_e                                   */
    int32_t rics_backend;     /* PIC1D_RICS_*                                */
    int32_t table_nlg;        /* TABLE: nodes in log10 gamma over [0, 8],    */
                              /*   2..4096; table_nlg * table_ns <= 2^27     */
    int32_t table_ns;         /* TABLE: nodes in s, 2..65536                 */
    int32_t pairs;            /* 1: photons with E >= 2 m_e c^2 make pairs   */
    int32_t conversion;       /* PIC1D_CONV_*                                */
    int32_t atmosphere;       /* 1: refill the surface layers (Appendix B.1) */
    int32_t gravity;          /* 1: gravity T/h towards the wall in the layer */
    int32_t frozen_field;     /* 1: skip Ampere (test mode)                  */
    int32_t annihilation;     /* 1: e-/e+ pairs annihilate in cells over n_max
                               *   (Sec. 3): see pic1d_step                   */
    int32_t photon_field;     /* PIC1D_FIELD_*: where the thermal photons come from */
    double nmax_over_n0;      /* n_max/n0 per cell, all species; <= 0: d0_cells^2 */
    double atm_a0;            /* peak atmosphere density / n0; <= 0: 18 |j_twist| */
    double atm_h_cells;       /* scale height in cells; <= 0: 3 d0 / a0^(1/2) */
    double atm_T;             /* atmosphere temperature / m_e c^2 (0.01)     */
    double atm_cut;           /* layer where a0 exp(-d/h) >= atm_cut (0.01)  */
    uint64_t seed;            /* Philox key                                  */
    int32_t sort_interval;    /* steps between cell sorts; 0 = never         */
    int32_t avg_start_step;   /* accumulate averages from this step; < 0 off */
    const float* mlp_weights; /* MLP backend: host, pic1d_mlp_param_count() fp32 parameters */
    const float* mlp_norm;    /* MLP backend: host, 6 floats: output mean[3], std[3] */
    double mlp_fallback_tol;  /* MLP backend: > 0 gives every line a RICS table and an error
                               *   estimate of the network on it -- the largest relative
                               *   error of F_hat and Ndot_hat against the closed forms
                               *   over the table's nodes (where they are significant:
                               *   |F| h >= 1e-9 max(u, 1), Ndot h >= 1e-9), evaluated on the
                               *   device at init -- and lines whose estimate exceeds the
                               *   tolerance use their table instead of the network;
                               *   any R_max and field range are then accepted.
                               *   0: the network everywhere (R_max = 4 lines only). */
    void* workspace;          /* device, >= pic1d_workspace_size bytes, 256-B aligned */
    size_t workspace_bytes;
    void* stream;             /* hipStream_t all work is enqueued on          */
} pic1d_config;

typedef struct {
    /* caller-owned host arrays; any may be NULL to skip it.  Sizes for a line
     * of n cells: n_cell[s] n, j n, E n, pair_rate n. */
    double* n_cell[4];        /* density per cell in units of n0, per species */
    double* j;                /* plasma current on cell centres, units n0 e c */
    double* E;                /* E on cell centres, code units                 */
    double* pair_rate;        /* pairs created per cell per step               */
    /* scalars always filled */
    double gauss_residual;    /* max_i |E_{i+1/2}-E_{i-1/2}-4 pi rho_i| / (4 pi Q ppc0), interior nodes */
    double v_circuit;         /* e V_c / m_e c^2 = -(1/c^2) sum_k E_k         */
    double energy_kinetic;    /* sum m c^2 (gamma - 1), code units            */
    double energy_field;      /* sum E^2 / 8 pi, code units                   */
    int64_t count[4];         /* live particles per species                   */
    int64_t counters[16];     /* PIC1D_CNT_* since init (slots 14-15 reserved) */
    int64_t step;             /* steps taken since init                       */
    int64_t avg_steps;        /* steps in the averages                        */
} pic1d_moments_out;

typedef struct pic1d_state pic1d_state;

/* Bytes of device workspace needed by cfg (cfg->workspace may be NULL).
 * Errors: EINVAL for an invalid config. */
int pic1d_workspace_size(const pic1d_config* cfg, size_t* bytes);

/* Build the state: geometry node tables and RICS tables on the host in FP64
 * (Appendix B.2), carve cfg->workspace, upload, and create the initial plasma
 * (Philox-uniform offsets, stratified ppc_init per cell).  cfg and the arrays
 * it points to are copied; the workspace stays owned by the caller and must
 * outlive the state.  *out receives the handle (NULL on error).
 * Errors: EINVAL (config), ENOMEM (workspace too small), EDEVICE. */
int pic1d_init(const pic1d_config* cfg, pic1d_state** out);

/* Advance all lines by n_steps >= 0 steps; enqueues the work and returns after
 * checking the device error word of the completed steps (this synchronises
 * the stream once per call).
 *
 * One step (Sec. 3): gather, RICS drag / events, kick, move, charge-conserving
 * deposit; photon conversion into pairs; atmosphere refill; with
 * cfg->annihilation, pair annihilation at the density limit; Ampere.  The
 * annihilation reading (the paper gives no mechanics): a cell holding N > n_max
 * particles of all species after the step's appends loses
 * k = min(N-, N+, ceil((N - n_max)/2)) e-/e+ pairs of species 0/1, those with
 * the smallest 64-bit Philox keys (step, id, stream 7), ties by id; the cell's
 * face current gains Q (sum x- - sum x+), as if each positron moved to its
 * electron before the neutral pair vanished, so Gauss's law holds.
 * Errors: ECAPACITY, ENONFINITE (state frozen), ESTATE, EDEVICE. */
int pic1d_step(pic1d_state* st, int32_t n_steps);

/* Diagnostics of one line (the quantities the paper's results are stated in):
 *   - per-cell densities of each species, the plasma current and E (Sec. 4.1 and
 *     Fig. 2: densities, multiplicity n e c / j, the field along the line), and
 *     the pairs created per cell per step (the pair-production rate of Sec. 4.1,
 *     Figs. 2-3), each instantaneous (the last step) or averaged over the steps
 *     since avg_start_step or the last RESET (the paper averages over
 *     ct/L in [5, 10]);
 *   - the circuit potential e V_c / m_e c^2 = -(1/m_e c^2) e integral E dl
 *     (Sec. 1, the definition of V_c; Sec. 4.1 reports it), from the cell-centred
 *     E (one cell per unit length);
 *   - the Gauss residual of the 1D Gauss law dE/dl = 4 pi rho (Secs. 3 and 5),
 *     max over interior nodes of |E_{i+1/2} - E_{i-1/2} - 4 pi rho_i| / (4 pi Q ppc0),
 *     rho from cloud-in-cell weights of the stored positions;
 *   - the kinetic energy sum m c^2 (gamma - 1) and the field energy sum E^2 / 8 pi
 *     (code units; the energy ledger of Sec. 3's Ampere update);
 *   - live counts and the counters.
 * Every sum is reproducible to the bit under any particle order: charge and
 * kinetic energy in integer fixed point, E sums over cells in a fixed order.
 * flags: PIC1D_MOM_INSTANT or _AVERAGE, plus PIC1D_MOM_RESET to restart the
 * averages after reading.  out and the arrays it points to are caller-owned host
 * memory.  Synchronises the stream.
 * Errors: EINVAL (line out of range), EDEVICE. */
int pic1d_moments(pic1d_state* st, int32_t line, int32_t flags, pic1d_moments_out* out);

/* Release the state (not the workspace).  NULL is a no-op. */
void pic1d_free(pic1d_state* st);

/* Text of the last error on st (or of the last failed init when st is NULL);
 * valid until the next call on the same handle. */
const char* pic1d_last_error(const pic1d_state* st);

/* Copy the live particles of one species of one line to host arrays of
 * `capacity` entries (cell, offset, u, id); *count receives the number of live
 * particles (EINVAL and nothing copied if it exceeds capacity).  The order is
 * the library's storage order, which carries no meaning. */
int pic1d_get_particles(pic1d_state* st, int32_t line, int32_t species, int64_t capacity,
                        int64_t* count, int32_t* cell, float* offset, float* u, uint64_t* id);

/* Replace one species of one line by `count` particles from host arrays.
 * cell in [0, n_cells), offset in [0, 1).  Errors: EINVAL, ECAPACITY. */
int pic1d_set_particles(pic1d_state* st, int32_t line, int32_t species, int64_t count,
                        const int32_t* cell, const float* offset, const float* u,
                        const uint64_t* id);

/* Copy E of one line (n_cells doubles) to / from host memory. */
int pic1d_get_field(pic1d_state* st, int32_t line, double* E);
int pic1d_set_field(pic1d_state* st, int32_t line, const double* E);

/* Set the step counter (keys the Philox draws); for restoring saved states. */
int pic1d_set_step(pic1d_state* st, int64_t step);

/* Per-kernel timing with HIP events.  pic1d_profile(st, 1) resets the totals
 * and records an event pair around every kernel that pic1d_step launches from
 * then on; pic1d_profile(st, 0) stops.  pic1d_profile_read fills out->ms[k]
 * (total milliseconds) and out->launches[k] for k = PIC1D_KERNEL_*. */
enum { PIC1D_KERNEL_PUSH = 0,
       PIC1D_KERNEL_APPEND = 1,   /* pair conversion and atmosphere refill (one launch) */
       PIC1D_KERNEL_FIELD = 2, PIC1D_KERNEL_PLAN = 3, PIC1D_KERNEL_SORT = 4,
       PIC1D_KERNEL_ANNIHILATE = 5,   /* annihilation plan and candidates (two launches) */
       PIC1D_NKERNELS = 8 };
typedef struct {
    double ms[8];
    int64_t launches[8];
} pic1d_profile_out;
int pic1d_profile(pic1d_state* st, int32_t enable);
int pic1d_profile_read(pic1d_state* st, pic1d_profile_out* out);

/* Capture the step sequence in HIP graphs of steps_per_graph steps (rounded up
 * to a multiple of sort_interval) and replay them in pic1d_step; 0 returns to
 * eager launches.  Graphs are captured on first use (one per live particle
 * buffer set) on a private stream and replayed on the config's stream; steps
 * before the next multiple of the graph length, remainders and profiled steps
 * run eagerly.  The results are the same as eager stepping.
 * Errors: EINVAL. */
int pic1d_set_graph(pic1d_state* st, int32_t steps_per_graph);

typedef struct {
    int32_t push_blocks_per_cu;  /* blocks of the particle kernel per compute unit */
    int32_t xcd_walk;            /* 1: tiles walked in one contiguous range per XCD */
    int32_t sort_interval;       /* steps between cell sorts                       */
    int32_t n_trials;            /* launch shapes timed                            */
    double ms_per_step_before;   /* with the shape the state had                   */
    double ms_per_step_after;    /* with the chosen shape                          */
    int32_t push_ppt;            /* particles per lane of a particle-kernel tile   */
    int32_t deposit_window;      /* cells of a wavefront's LDS deposit window      */
    int32_t sort_granularity;    /* sort bins per cell                             */
} pic1d_tune_out;

/* Autotuner of the launch shape: times trial_steps real steps (at least one
 * sort cycle) for each candidate -- the particle kernel's tile shape (4, 8 or
 * 16 particles per lane; the deposit window, 128 cells for the TABLE backend,
 * 32 or 64 for OFF and EXACT, wherever that shape is built: never below the
 * backend's default, which holds a tile's particles once a heated plasma spreads
 * them between sorts), push
 * blocks per CU in {1,2,3,4,6,8}, the XCD-aware tile walk on/off, sort_interval
 * in {1,2,5,10,25,50,100}, then (when sorting) 8, 16 or 32 sort bins per cell
 * -- one knob at a time, and keeps the fastest; a tile shape, block count or
 * sort granularity other than the starting one must beat it again when the two
 * are timed alternately twice.  The trial steps advance the simulation; the
 * physics does not depend on these choices (particle order and launch shape do
 * not change any result).  Errors: EINVAL, ESTATE, ECAPACITY, ENONFINITE. */
int pic1d_autotune(pic1d_state* st, int32_t trial_steps, pic1d_tune_out* out);

/* Set the particle kernel's launch shape directly: blocks per CU (1..32),
 * particles per lane of a tile (4, 8, 16) and the deposit window in cells (the
 * combinations pic1d_autotune lists, and a 64-cell window for the TABLE
 * backend; the MLP backend has 8 and 32 only).  The results do not depend on
 * it.  Errors: EINVAL (a shape that is not built), ESTATE. */
int pic1d_set_push_shape(pic1d_state* st, int32_t blocks_per_cu, int32_t ppt, int32_t window);

/* Granularity of the cell sort: after a sort every species' particles are in
 * nondecreasing order of cell * bins_per_cell + min(floor(offset *
 * bins_per_cell), bins_per_cell - 1) (8 on a new state; a power of two, 1 to
 * 32).  Finer bins group the particles that cross a cell face more tightly in
 * memory at a higher counting cost.  The results do not depend on it.  Waits
 * for the stream and drops captured graphs.  Errors: EINVAL, ESTATE. */
int pic1d_set_sort_granularity(pic1d_state* st, int32_t bins_per_cell);

/* The surrogate's error estimate on one line and whether the line uses its
 * table instead (MLP backend with mlp_fallback_tol > 0; otherwise *error = -1 and
 * *uses_table = 1 for the TABLE backend, 0 for the others).  Host outputs.
 * Errors: EINVAL. */
int pic1d_rics_line_info(pic1d_state* st, int32_t line, double* error, int32_t* uses_table);

/* Evaluate the configured RICS backend of one line at n points, exactly as
 * the pusher does (float32): device arrays s_cells[n] (arc length in cells,
 * geometry interpolated from the nodes) and u[n]; outputs device arrays
 * F[n] (F_hat), ndot[n] (Ndot_hat), eps[n] (photon energy / m_e c^2).
 * Errors: EINVAL. */
int pic1d_rics_eval(pic1d_state* st, int32_t line, int64_t n, const float* s_cells,
                    const float* u, float* F, float* ndot, float* eps);

/* ---------------------------------------------------------------------------
 * Test-particle map of the magnetosphere (Appendix A.4, Fig. 6).
 *
 * For each field line of equatorial radius r_eq[k] (in R*), a lepton is injected
 * at the northern footpoint with Lorentz factor gamma0, moving away from the
 * star, and moves under the RICS drag force of Eq. contdrag alone (radial beam,
 * no electric field).  One device thread per line integrates
 *   dv/dt = -beta / (R (1 + 3 v^2)^(1/2)), du/dt = F_hat, dN/dt = Ndot_hat
 * (v = cos theta, t in units of R* over c) by fourth-order Runge-Kutta in float64 with the
 * step limited by tol_stiff / |dF/du|, tol |u| / |F|, tol / Ndot, tol |v| / |dv/dt|
 * and dt_max, until the particle crosses the equator or t_max L / c.
 * Results per line (lengths in R* of arc from the northern footpoint):
 *   gamma_min  the lowest gamma on the way to the equator (at the crossing, or
 *              over the integration time when the drag holds the particle near
 *              its attractor beta = mu -> 0 at the equator);
 *   s_first    where the expected number of scatterings reaches 1 (-1: never);
 *   s_b        where b first drops below b_pp (-1: b >= b_pp on the whole line);
 *   l_pp       the pair-production zone, s_b - s_first, or L - 2 s_first when the
 *              line never reaches b < b_pp (the zone then spans the equator,
 *              taken symmetric about it), 0 without a first scattering;
 *   crossed    1 if the particle crossed the equator.
 * ------------------------------------------------------------------------- */
typedef struct {
    double gamma0;            /* injection Lorentz factor (1000 in Fig. 6)   */
    double kT_keV;            /* photon temperature (1 keV in Fig. 6)        */
    double b_pole;            /* B* / B_QED (10)                             */
    double b_pp;              /* pair threshold (0.1)                        */
    double t_max;             /* integration time in units of L / c (4)      */
    double dt_max;            /* largest step, units of R* over c (1e-2)     */
    double tol;               /* relative change per step (1e-3)             */
    double tol_stiff;         /* |dF/du| dt per step (0.3; RK4 is stable below 2.78) */
    int64_t max_steps;        /* per line (1e8)                              */
} pic1d_tp_config;

typedef struct {
    double gamma_min, s_first, s_b, l_pp, L;
    int32_t crossed, pad;
    int64_t steps;            /* Runge-Kutta steps taken                     */
} pic1d_tp_result;

/* Device workspace of a sweep over n lines. */
int pic1d_testparticle_workspace_size(int32_t n, size_t* bytes);

/* Sweep n >= 1 lines: r_eq (host, n values > 1), out (host, n results); the
 * workspace (device, 256-byte aligned) holds the device copies.  Synchronises
 * the stream.  Errors: EINVAL, ENOMEM (workspace), EDEVICE. */
int pic1d_testparticle_sweep(const pic1d_tp_config* cfg, int32_t n, const double* r_eq, pic1d_tp_result* out,
                             void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * RICS surrogate network (RICS backend PIC1D_RICS_MLP).
 *
 * The paper evaluates the RICS drag force and scattering rate from their
 * definitions (Sec. 2.2, Eqs. scatteringNdot and contdrag) and proposes no
 * surrogate; this network is an addition trained on those definitions.
 * Inputs (log10 gamma, s/L, log10(B/B_QED), kT/keV) on [0,8] x [0,1] x [-2,3] x
 * [0.3,1], s/L along the R_max = 4 dipole line (Appendix B.2); network
 * 4 -> 128 -> 128 -> 128 -> 128 -> 3 with SiLU; outputs the normalised targets
 * (o_k - mean_k)/std_k of o1 = log10(|F_hat|/|gamma mu - u|), o2 = log10(Ndot_hat),
 * o3 = log10(eps) (Appendix A.3) for u >= 0; negative u by the mirror
 * F(-u, s) = -F(u, L - s).  Weights run on the matrix cores in bfloat16 with
 * float32 accumulation (activations as three bfloat16 terms).
 *
 * Parameters: PIC1D_MLP_NPARAM floats, [W1 (128x4, row-major), b1, W2 (128x128),
 * b2, W3, b3, W4, b4, W5 (3x128), b5].  Inputs x: n x 4 floats (raw, not
 * normalised); targets o: n x 4 floats (o1, o2, o3, 0).  Device pointers must be
 * 16-byte aligned; workspaces 256-byte aligned.  Stateless calls report errors
 * through pic1d_last_error(NULL).
 * ------------------------------------------------------------------------- */
#define PIC1D_MLP_NPARAM 50563

int pic1d_mlp_param_count(void);

/* Device workspace for a batch of `batch` samples and a training pool of
 * n_pool samples (0 for forward / loss_grad only). */
int pic1d_mlp_workspace_size(int64_t batch, int64_t n_pool, size_t* bytes);

/* Samples first .. first+n-1 of the seeded sample stream: sample i takes the
 * first Philox block (counter (i_lo, i_hi, attempt, 7), key = seed) whose
 * inputs log10 gamma = 8 U0, s/L = U1, log10 b = -2 + 5 U2, kT = 0.3 + 0.7 U3
 * lie within the Planck cutoff y <= 80; targets in float64, stored float32.
 * x, o: device, n x 4 floats.  workspace: device, 256-byte aligned, at least
 * PIC1D_MLP_SAMPLES_WORKSPACE bytes (the kernel's error word; the call allocates
 * nothing).  Synchronises the stream.
 * Errors: EINVAL, ENOMEM (workspace), ENONFINITE (a sample found no accepted draw). */
#define PIC1D_MLP_SAMPLES_WORKSPACE 256
int pic1d_mlp_samples(uint64_t seed, int64_t first, int64_t n, float* x, float* o, void* workspace,
                      size_t workspace_bytes, void* stream);

/* Network outputs (normalised targets, n x 3 floats, device) for raw inputs x
 * (device, n x 4) with parameters `params` (device, fp32).  Synchronises.
 * Errors: EINVAL, ENOMEM (workspace), EDEVICE. */
int pic1d_mlp_forward(const float* params, int64_t n, const float* x, float* out, void* workspace,
                      size_t workspace_bytes, void* stream);

/* Mean squared error of the network outputs against normalised targets t
 * (device, n x 3) and its gradient with respect to the bfloat16-rounded weights
 * and the biases (grad: device, PIC1D_MLP_NPARAM floats); *loss (host) may be
 * NULL.  Synchronises.  Errors: EINVAL, ENOMEM, EDEVICE. */
int pic1d_mlp_loss_grad(const float* params, int64_t n, const float* x, const float* t, float* grad,
                        double* loss, void* workspace, size_t workspace_bytes, void* stream);

/* pic1d_mlp_loss_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with no workspace argument.  The
 * batch's activations and partial sums live in a static device array of 12 MiB
 * that each GPU the library runs on holds until the process ends (its address
 * taken once per device).  n <= 2048 samples (EINVAL beyond).  Every call on one
 * GPU shares that array: calls that overlap on one GPU (two host threads, or
 * two streams) race and must not be made; each call fully rewrites what it
 * reads.  Allocates nothing; synchronises the stream when loss != NULL.
 * Errors: EINVAL, EDEVICE. */
int pic1d_mlp_loss_grad_static(const float* params, int64_t n, const float* x, const float* t, float* grad,
                               double* loss, void* stream);

/* One Adam step (Kingma & Ba 2015, Algorithm 1) on device arrays of
 * PIC1D_MLP_NPARAM floats; t >= 1 is the step number.  Synchronises. */
int pic1d_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t t, double lr, double beta1,
                   double beta2, double eps, void* stream);

typedef struct {
    uint64_t seed;            /* sample stream, initial weights and batches */
    int64_t n_samples;        /* training pool: samples 0 .. n_samples-1 of the stream */
    int32_t batch;            /* samples per Adam step, drawn with replacement */
    int32_t steps;            /* Adam steps                                   */
    double lr, lr_final;      /* cosine schedule from lr to lr_final          */
    double beta1, beta2, eps; /* Adam constants; <= 0 selects 0.9, 0.999, 1e-8 */
    const float* init_params; /* host initial parameters, or NULL for Glorot-uniform weights from seed */
    void* workspace;          /* device, >= pic1d_mlp_workspace_size(batch, n_samples) */
    size_t workspace_bytes;
    void* stream;
} pic1d_mlp_train_config;

typedef struct {
    float* params;            /* host out: PIC1D_MLP_NPARAM floats            */
    float* norm;              /* host out: mean[3], std[3] of the targets      */
    double* loss;             /* host out (optional): loss at n_loss evenly spaced steps */
    int32_t n_loss;           /* in: capacity of loss; out: entries written   */
    double loss_first, loss_last;
    double seconds;           /* wall time of the call                        */
} pic1d_mlp_train_result;

/* Train the network on the GPU: draw the sample pool, normalise the targets by
 * their mean and standard deviation, then `steps` Adam steps on batches drawn
 * from the pool, each a forward, backward and weight-gradient pass on the
 * matrix cores.  Errors: EINVAL, ENOMEM, EDEVICE, ENONFINITE. */
int pic1d_mlp_train(const pic1d_mlp_train_config* cfg, pic1d_mlp_train_result* res);

#ifdef __cplusplus
}
#endif

#endif /* PIC1D_H */
