/*
 * pc.h -- C ABI of the MI355X (gfx950) 1D PIC-MCC positive-column library.
 *
 * The library advances a one-dimensional electrostatic Particle-In-Cell /
 * Monte Carlo Collisions model of a neon or argon positive column: electrons
 * and positive ions on a uniform grid, field from Poisson's equation every
 * step, electron-atom elastic / lumped-excitation / ionization collisions and
 * ion-atom charge exchange by the null-collision method, radial losses as a
 * per-particle removal frequency (Boeuf, "Ionization waves (striations) in a
 * low-current plasma column revisited with kinetic and fluid models",
 * section II for the model, eq. (2) for the radial losses, section V for the
 * bounded column).
 *
 * Conventions
 *  - Every function returns a pc_status: PC_OK (0) or a negative error code.
 *    No C++ exception crosses this boundary.  pc_last_error() returns a
 *    thread-local human-readable detail for the last failure.
 *  - Device memory is owned by the caller.  pc_init_column receives one
 *    workspace of pc_sizes.workspace_bytes bytes (256-byte aligned) and lays
 *    out all particle arrays, charges, fields and counters inside it; the
 *    library never allocates device memory.  Output arrays are caller-owned
 *    device buffers as documented per function.
 *  - All work is enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*).  Functions marked "async" return before the work completes;
 *    pc_sync / pc_get_counts wait for the stream and surface device-side
 *    errors.  After a device-side error the handle is poisoned: further
 *    pc_step calls return PC_ERR_POISONED until pc_set_state clears it.
 *  - Particle state is exchanged as structure-of-arrays, FP64: x [m] in
 *    [0, L), vx, vy, vz [m/s] (vx is the leapfrog half-step velocity), id
 *    (uint32).  FP32 columns store (cell, offset in [0,1), velocities in cells
 *    per step) internally and convert at the state entry points.  Node
 *    arrays have pc_sizes.n_nodes entries: n_cells + 1 (bounded) or n_cells
 *    (periodic).  Charges are int64 fixed point with 25 fractional bits: a
 *    macroparticle contributes exactly 2^25 units split between its two
 *    nodes.
 */
#ifndef PC_H
#define PC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pc_status;
enum {
    PC_OK = 0,
    PC_ERR_INVALID_ARG = -1,     /* null pointer, bad size, bad enum */
    PC_ERR_UNSTABLE_CONFIG = -2, /* violates dt < 0.2/w_pe, dx < lambda_De, nu_max dt <= 0.1 */
    PC_ERR_CAPACITY = -3,        /* particle, birth or loss list capacity exceeded */
    PC_ERR_NONFINITE = -4,       /* a position left [0, L) after the boundary rule, or NaN */
    PC_ERR_ECAP = -5,            /* electron energy above eps_cap / frequency above nu_max */
    PC_ERR_GCAP = -6,            /* ion-atom relative speed above g_cap */
    PC_ERR_HIP = -7,             /* a HIP runtime call failed */
    PC_ERR_POISONED = -8,        /* an earlier device-side error is pending */
    PC_ERR_WORKSPACE = -9,       /* workspace too small or misaligned */
    PC_ERR_IDS = -10             /* particle id space (2^32) exhausted */
};

enum { PC_BOUNDED = 0, PC_PERIODIC = 1 };
/* radial sink: off; fixed frequency nu_w (eq. (2)); balanced: each particle
 * is removed with probability (ionizations since the species' previous step)
 * / (its count), keeping the particle number constant on average as the
 * paper's removal of one electron-ion pair per ionization does (section II);
 * pair: the paper's model itself -- per ionization one electron and one ion,
 * each drawn uniformly among the live ones of its species, are removed
 * before the field solve and the products take their slots and ids (the
 * counts stay constant; periodic columns only, ids a permutation of
 * 0..n-1, at most 2048 ionizations per step; single columns, not batches) */
enum { PC_WALL_OFF = 0, PC_WALL_FIXED = 1, PC_WALL_BALANCED = 2, PC_WALL_PAIR = 3 };
enum { PC_SHARE_OPB = 0, PC_SHARE_EQUAL = 1 };
enum { PC_ELECTRON = 0, PC_ION = 1 };
enum { PC_FP64 = 0, PC_FP32 = 1 };
/* event codes written by pc_step into the optional per-id event buffers */
enum { PC_EV_NONE = 0, PC_EV_ELASTIC = 1, PC_EV_EXCITE = 2, PC_EV_IONIZE = 3,
       PC_EV_WALL = 4, PC_EV_ABSORB = 5, PC_EV_CX = 6, PC_EV_NULL = 7 };

/* Column description (SI units unless noted).  Cross sections are the
 * synthetic analytic forms: elastic A + B eps^p (p = +-1/2, eps in eV),
 * excitation and ionization 4 smax (U/eps)(1 - U/eps) above threshold U [eV],
 * constant charge exchange.  V is the anode potential (bounded) or E0 L
 * (periodic, imposed mean field E = -E0 + E_sp, section II). */
typedef struct pc_config {
    int32_t bc, n_cells, ppc, ion_subcycle;
    int32_t wall_mode, energy_sharing, poisson, sort_interval;
    int32_t launch_blocks;   /* blocks of the particle kernels (0 = auto: one initial particle
                                per thread, at most 4096 blocks) */
    int32_t precision;       /* PC_FP64: FP64 particle state; PC_FP32: FP32 cell-relative
                                state and push (field solve and collision arithmetic FP64) */
    int32_t pad1, pad2;
    double L, V, p_torr, Tg, n0, Te0_eV, Ti0_K, nu_w, dt, eps_cap, g_cap, capacity;
    double M_amu, el_A, el_B, el_p, ex_U, ex_smax, iz_U, iz_smax, cx_sigma, opb_w;
    /* bounded columns (section V): cathode emission current density emit_J
     * [A/m^2] (0 = none) of electrons at temperature emit_T [eV]; series
     * resistance circuit_R [ohm m^2] between the source V and the anode
     * (0 = anode held at V).  Single columns only. */
    double emit_J, emit_T, circuit_R;
    uint64_t seed;
} pc_config;

typedef struct pc_sizes {
    int64_t workspace_bytes; /* bytes the caller must provide */
    int64_t capacity;        /* particle slots per species */
    int64_t max_births;      /* ionizations per step */
    int64_t max_losses;      /* losses per species per step */
    int32_t n_nodes, n_cells;
    double nu_max;           /* null-collision bound of the electrons [1/s] */
    double p_null;           /* electron collision-candidate probability per step */
    double p_cx;             /* ion candidate probability per ion step */
} pc_sizes;

typedef struct pc_counts {
    int64_t n[2];            /* live particles per species */
    int64_t next_id[2];      /* next id per species */
    int64_t step;            /* index of the next step */
    uint32_t errors;         /* sticky device error bits */
    uint32_t pad;
    int64_t births_last;     /* ionizations of the previous step (balanced sink) */
    int64_t births_since_ion; /* ionizations since the last ion step (balanced sink) */
    double V_anode;          /* anode potential of the last field solve [V] (circuit) */
    double J_cond;           /* conduction current density of the last step [A/m^2] */
    int64_t vsum_ion;        /* ions' sum of v_x at their last step, 2^-20 m/s units */
    double emit_carry;       /* fraction of an emitted electron carried to the next step */
} pc_counts;

typedef struct pc_column* pc_handle;

/* Sizes of the workspace and lists for a config.  Validates the config. */
pc_status pc_query_sizes(const pc_config* cfg, pc_sizes* out);

/* Create a column in the caller's workspace and load it (async): uniform
 * positions, Maxwellian velocities (electrons at Te0, ions at Ti0), ids
 * 0..N0-1, deposit, field solve and the leapfrog half-step back of vx
 * (section II: uniform and equal initial densities).  Rejects configs that
 * break dt < 0.2/w_pe or dx < lambda_De (section II) or nu_max dt <= 0.1. */
pc_status pc_init_column(const pc_config* cfg, void* workspace, size_t bytes,
                         void* hip_stream, pc_handle* out);

/* Advance n_steps full time steps (async).  Per step: electrons (CIC gather,
 * leapfrog push, boundary, radial sink, null-collision MCC, fused fixed-point
 * deposit), ions every ion_subcycle steps with dt_i = ion_subcycle dt,
 * removal of losses, append of ionization products (ids by rank of the
 * parent id), field solve; a per-cell counting sort every sort_interval
 * steps (no effect on results).  On a non-null stream the steps are replayed
 * from HIP graphs: whole periods of lcm(2, 2 ion_subcycle, 4 sort_interval)
 * steps (after which every buffer parity returns) and the remainder of
 * n_steps each as one graph, captured the first time a (phase, length) is
 * met and cached (at most 64 graphs per column, least recently used
 * dropped).  Event buffers or an enabled kernel timer make the launches
 * eager.  Results are bitwise identical either way. */
pc_status pc_step(pc_handle h, int64_t n_steps);

/* Capture, without executing anything, the graphs that a following
 * pc_step(h, n_steps) will replay, so that its launches carry no capture
 * cost (blocking on the host only; the column's state is unchanged). */
pc_status pc_prepare_graphs(pc_handle h, int64_t n_steps);

/* Deposit n positions (device FP64, all in [0, L)) with linear weighting
 * into rho (device int64[n_nodes], overwritten).  Async. */
pc_status pc_deposit(pc_handle h, const double* x, int64_t n, int64_t* rho);

/* Solve Poisson's equation (section II) for node charges rho_e, rho_i (device
 * int64[n_nodes]) into E (device double[n_nodes]) and, if phi is non-null,
 * phi (device double[n_nodes]).  Bounded: phi(0) = 0, phi(L) = V.  Periodic:
 * mean charge neutralised, phi(0) = 0, E = -E0 + E_sp.  Async. */
pc_status pc_solve_field(pc_handle h, const int64_t* rho_e, const int64_t* rho_i,
                         double* phi, double* E);

/* Cell moments of the current state into out (device int64, async), layout
 * with nc = n_cells: [0,nc) electron count, [nc,2nc) sum eps 2^20 (eV),
 * [2nc,3nc) sum vx 2^10, [3nc,4nc) sum eps vx 2^4, [4nc,5nc) ion count,
 * [5nc,6nc) ion sum vx 2^10, [6nc,7nc) ionizations since the last reset,
 * then ceil(nc/cells_per_group) x 240 EEPF counts (0.25 eV bins on
 * [0, 60) eV).  Each term is truncated to an integer per particle. */
pc_status pc_moments(pc_handle h, int32_t cells_per_group, int32_t reset_iz, int64_t* out);

/* Synchronise the stream and read the counters (blocking). */
pc_status pc_get_counts(pc_handle h, pc_counts* out);

/* Copy the first n live particles of a species into caller device arrays
 * (any pointer may be null; cap = array length).  Async; n from pc_get_counts. */
pc_status pc_get_state(pc_handle h, int32_t species, double* x, double* vx, double* vy,
                       double* vz, uint32_t* id, int64_t cap);

/* Replace a species' particles with n caller device arrays (async).  Clears
 * a poisoned handle.  Positions must lie in [0, L).  For the ions, the charge
 * held between ion steps is redeposited from the new particles. */
pc_status pc_set_state(pc_handle h, int32_t species, int64_t n, const double* x,
                       const double* vx, const double* vy, const double* vz,
                       const uint32_t* id);

/* Set the step index and next ids (blocking). */
pc_status pc_set_counters(pc_handle h, int64_t step, int64_t next_e, int64_t next_i);
/* External circuit and emission state (section V), for restarts and parity
 * checks (blocking): anode potential, the ions' held v_x sum (as in
 * pc_counts) and the emission carry. */
pc_status pc_set_circuit(pc_handle h, double V_anode, int64_t vsum_ion, double emit_carry);

/* Set the ionization tallies of the balanced sink (blocking). */
pc_status pc_set_balance(pc_handle h, int64_t births_last, int64_t births_since_ion);

/* Copy the current field E^n and the charges it was solved from (async;
 * any pointer may be null). */
pc_status pc_get_field(pc_handle h, double* E, int64_t* rho_e, int64_t* rho_i);
/* Overwrite the current field E^n (async). */
pc_status pc_set_field(pc_handle h, const double* E);

/* Optional per-id event recording for parity checks: device uint8 buffers
 * indexed by particle id; each step writes the event code of every particle
 * it advances (ids >= len are skipped).  Null disables. */
pc_status pc_set_events(pc_handle h, uint8_t* ev_e, int64_t len_e, uint8_t* ev_i,
                        int64_t len_i);

/* Kernel timer for roofline measurements: with max_launches > 0, pc_step
 * times each launch of the electron advance kernel (the dominant kernel:
 * gather, push, collisions, deposit) with a pair of HIP events that take the
 * start and end timestamps of the launch itself (hipExtLaunchKernelGGL), up
 * to max_launches launches (launches are then eager, not graph-replayed).  The event pool is created here, never inside pc_step;
 * 0 disables the timer and frees the pool. */
pc_status pc_timer_enable(pc_handle h, int64_t max_launches);
/* Wait for the recorded launches and return their summed duration [ms] and
 * count; resets the timer for the next window (blocking). */
pc_status pc_timer_read(pc_handle h, double* total_ms, int64_t* launches);

/* Synchronise the stream and map device error bits to a status. */
pc_status pc_sync(pc_handle h);

/* Free the host-side handle (the workspace stays with the caller). */
void pc_destroy(pc_handle h);

/* ------------------------------------------------------------------ batch
 * Many independent columns advanced together (the parameter scans of
 * sections III and V run as one job).  Each step is one launch over the
 * particle chunks of every column, ions on subcycle steps, and one finish
 * workgroup per column (field, births, losses); the whole period is
 * replayed as one HIP graph.  Columns keep their own configs, seeds, ids and
 * buffers, and a batch column evolves bitwise exactly as the same column
 * stepped alone with pc_step.  Columns may differ in every field except
 * precision, ion_subcycle and sort_interval, which the batch shares. */
typedef struct pc_batch* pc_batch_handle;

typedef struct pc_tuning {
    int32_t chunk;           /* particles per workgroup item of the particle launches */
    int32_t sort_interval;   /* steps between counting sorts (0 = never) */
    int32_t n_items_e, n_items_i; /* workgroups per electron / ion launch */
    double us_per_step;      /* measured by pc_batch_tune, else 0 */
} pc_tuning;

/* Workspace bytes for n_columns configs (validates every config). */
pc_status pc_query_batch_sizes(const pc_config* cfgs, int32_t n_columns, int64_t* workspace_bytes);

/* Create and load n_columns columns in one workspace (async, as
 * pc_init_column for each). */
pc_status pc_init_batch(const pc_config* cfgs, int32_t n_columns, void* workspace, size_t bytes,
                        void* hip_stream, pc_batch_handle* out);

/* Advance every column by n_steps (async). */
pc_status pc_batch_step(pc_batch_handle b, int64_t n_steps);

/* Borrowed handle of column c for the per-column calls (state, counts,
 * field, moments, deposit, solve).  pc_step, pc_set_events and the kernel
 * timer reject it; pc_destroy ignores it (pc_batch_destroy frees it). */
pc_status pc_batch_column(pc_batch_handle b, int32_t column, pc_handle* out);

/* Autotuner: times trial_steps real steps for each chunk size in {1024,
 * 2048, 3072, 4096, 6144, 8192} and sort interval in {10, 20, 40, 80}, keeps
 * the fastest (blocking).  No setting changes any result. */
pc_status pc_batch_tune(pc_batch_handle b, int32_t trial_steps, pc_tuning* out);
pc_status pc_batch_get_tuning(pc_batch_handle b, pc_tuning* out);
/* chunk >= 256 particles per workgroup; sort_interval >= 0 */
pc_status pc_batch_set_tuning(pc_batch_handle b, int32_t chunk, int32_t sort_interval);

/* Kernel timer of the batched electron launch (as pc_timer_enable/read). */
pc_status pc_batch_timer_enable(pc_batch_handle b, int64_t max_launches);
pc_status pc_batch_timer_read(pc_batch_handle b, double* total_ms, int64_t* launches);

/* Synchronise and map every column's device error bits (blocking); the
 * first failing column poisons the batch. */
pc_status pc_batch_sync(pc_batch_handle b);

/* Free the batch and its member handles (the workspace stays with the caller). */
void pc_batch_destroy(pc_batch_handle b);

/* Stream probe (measurement, not part of the model): dst = src over n FP64
 * device elements (n <= 2^29, arrays must not overlap), with the access form
 * of the particle kernels -- each of `blocks` 256-thread workgroups (0 =
 * 4096) walks a contiguous chunk, one 8-byte element per lane -- so that its
 * bytes per second are the achievable rate of that form and its hardware
 * counters calibrate the particle kernels' counters.  Async on hip_stream. */
pc_status pc_stream_probe(const double* src, double* dst, int64_t n, int32_t blocks, void* hip_stream);

const char* pc_status_string(pc_status s);
const char* pc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
