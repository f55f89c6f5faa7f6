/*
 * pco.h -- plain FP64 CPU oracle of the 1D electrostatic PIC-MCC column step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header or constant table with the GPU
 * library: both are written independently from the paper (section II, the
 * PIC-MCC model) and from the readings listed in the design notes.
 *
 * Everything runs serially on host memory, in IEEE double precision, in the
 * step order: electrons (gather, push, boundary, radial sink, null-collision
 * MCC), ions on subcycle steps, removal of losses, append of ionization
 * products ordered by parent id, charge deposit, field solve.
 *
 * All functions return 0 on success and a negative code on error.
 */
#ifndef PCO_H
#define PCO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { PCO_BOUNDED = 0, PCO_PERIODIC = 1 };
enum { PCO_WALL_OFF = 0, PCO_WALL_FIXED = 1, PCO_WALL_BALANCED = 2, PCO_WALL_PAIR = 3 };
enum { PCO_SHARE_OPB = 0, PCO_SHARE_EQUAL = 1 };
enum { PCO_ELECTRON = 0, PCO_ION = 1 };

/* event codes recorded per particle id for the last step */
enum { PCO_EV_NONE = 0, PCO_EV_ELASTIC = 1, PCO_EV_EXCITE = 2, PCO_EV_IONIZE = 3,
       PCO_EV_WALL = 4, PCO_EV_ABSORB = 5, PCO_EV_CX = 6, PCO_EV_NULL = 7 };

/* error bits (sticky, returned by pco_errors) */
enum { PCO_ERR_ECAP = 1, PCO_ERR_GCAP = 2, PCO_ERR_NUMAX = 4, PCO_ERR_IDS = 8, PCO_ERR_BIRTHS = 32 };

/* pair sink: largest number of ionizations per step (victims are listed per step) */
#define PCO_PAIR_MAX_BIRTHS 2048

typedef struct pco_config {
    int32_t bc, n_cells, ppc, ion_subcycle;
    int32_t wall_mode, energy_sharing, poisson, pad0;
    double L, V, p_torr, Tg, n0, Te0_eV, Ti0_K, nu_w, dt, eps_cap, g_cap;
    double M_amu, el_A, el_B, el_p, ex_U, ex_smax, iz_U, iz_smax, cx_sigma, opb_w;
    /* bounded column of section V: cathode emission current density [A/m^2]
     * at temperature emit_T [eV]; series resistance [ohm m^2] to the source V */
    double emit_J, emit_T, circuit_R;
    uint64_t seed;
} pco_config;

typedef struct pco_column pco_column;

/* Philox4x32 with 10 rounds (Salmon et al., SC'11): out = bijection(ctr; key). */
void pco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* create a column (grid, constants, empty particle lists); NULL on bad config */
pco_column* pco_create(const pco_config* cfg);
void pco_destroy(pco_column* c);
/* load both species, deposit, solve, leapfrog half-step back */
int pco_init_column(pco_column* c);
/* advance n full time steps */
int pco_step(pco_column* c, int64_t n);

/* stand-alone deposit of arbitrary positions in [0, L) into int64 node charge */
int pco_deposit(const pco_column* c, const double* x, int64_t n, int64_t* rho);
/* stand-alone field solve (Thomas algorithm) from fixed-point node charges;
 * phi and E have n_nodes entries (phi may be NULL) */
int pco_solve_field(const pco_column* c, const int64_t* rho_e, const int64_t* rho_i,
                    double* phi, double* E);

int32_t pco_n_nodes(const pco_column* c);
int64_t pco_count(const pco_column* c, int species);
int64_t pco_step_index(const pco_column* c);
int64_t pco_next_id(const pco_column* c, int species);
uint32_t pco_errors(const pco_column* c);
/* threads of the OpenMP timing build (n > 0 sets them); 1 in the serial build */
int pco_threads(int n);
/* scalar derived constants: 0 dx, 1 nu_max, 2 P_null, 3 weight W, 4 Ng, 5 P_cx */
double pco_constant(const pco_column* c, int which);

int pco_get_state(const pco_column* c, int species, double* x, double* vx, double* vy,
                  double* vz, uint32_t* id);
int pco_set_state(pco_column* c, int species, int64_t n, const double* x, const double* vx,
                  const double* vy, const double* vz, const uint32_t* id);
/* set the step index and the next ids (used to start from a shared state) */
int pco_set_counters(pco_column* c, int64_t step, int64_t next_e, int64_t next_i);
/* balanced sink: ionizations of the previous step and since the last ion step */
int pco_set_balance(pco_column* c, int64_t births_last, int64_t births_since_ion);
int pco_get_balance(const pco_column* c, int64_t out[2]);
/* pair sink: ids removed by the last step (victim r of ionization rank r);
 * returns their number and copies at most cap of them */
int64_t pco_get_victims(const pco_column* c, int species, uint32_t* out, int64_t cap);
/* section V state: anode potential, ions' held v_x sum (2^-20 m/s units) and
 * the emission carry; get returns (V_anode, last conduction current density,
 * carry) and the ion sum */
int pco_set_circuit(pco_column* c, double V_anode, int64_t vsum_ion, double emit_carry);
int pco_get_circuit(const pco_column* c, double out[3], int64_t* vsum_ion);
/* current field E^n at nodes and the charges it came from */
int pco_get_field(const pco_column* c, double* E, int64_t* rho_e, int64_t* rho_i);
int pco_set_field(pco_column* c, const double* E);
/* events of the last step, indexed by id (entries >= next_id are left alone) */
int pco_get_events(const pco_column* c, int species, uint8_t* ev, int64_t len);

/* cell moments of the current state, int64 layout (nc = n_cells):
 *   [0,nc) electron count, [nc,2nc) sum eps*2^20 (eV), [2nc,3nc) sum vx*2^10,
 *   [3nc,4nc) sum eps*vx*2^4, [4nc,5nc) ion count, [5nc,6nc) ion sum vx*2^10,
 *   [6nc,7nc) ionizations since the last reset,
 *   then n_groups*240 EEPF counts (0.25 eV bins on [0,60) eV) per group of
 *   cells_per_group cells.                                                   */
int pco_moments(pco_column* c, int32_t cells_per_group, int32_t reset_iz, int64_t* out);

#ifdef __cplusplus
}
#endif
#endif
