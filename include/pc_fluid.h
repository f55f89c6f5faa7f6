/*
 * pc_fluid.h -- C ABI of the batched quasi-neutral fluid column (gfx950).
 *
 * The fluid model of section IV of the paper (Boeuf): electron continuity
 * (3) and energy (4) equations with Joule heating (5), drift-diffusion
 * fluxes (12)-(13) with the coefficients (14)-(16) of temperature-dependent
 * transport coefficients (eq. (9) read as beta = 3/2 T mu_eps and
 * G = 3/2 T D_eps), and the quasi-neutral field (17) in a periodic column
 * with an imposed mean field E0 (which fixes the constant total flux).  The
 * closure fluxes come either from eqs. (12)-(13) with tabulated coefficients
 * (0D Boltzmann tables) or from the closure network of pc_mlp.h.
 *
 * Discretisation: N cells (a power of two, 64..4096), periodic finite
 * volumes; face values from the means of the two cells, coefficients by
 * linear interpolation in T (clamped to the table); backward Euler for the
 * diffusion of density (coefficient D_a) and of energy density (kappa, with
 * T' = w'/(1.5 n')), everything else explicit; floors n >= n_floor,
 * T >= T_min.  State and fluxes in FP32, the two cyclic tridiagonal systems
 * per column and step in FP64 (cyclic reduction in LDS).
 *
 * Table: table_len rows (2..1024) on T_k = T_min + k T_step [eV], 6 columns:
 *   mu_e N [1/(V m s)], D_e N [1/(m s)], mu_eps N, D_eps N, k_iz [m^3/s]
 *   (nu_i = N k_iz), L/N [eV m^3/s] (collisional energy loss per electron).
 * State: n [m^-3] and w = 3/2 n T [eV m^-3], device float [n_columns][n_cells].
 * Network closure inputs per face (n_f, 3/2 T_f, E_f, dn/dx, d(3/2 T)/dx) are
 * normalised as (v - norm[k]) * norm[5 + k]; outputs give
 * Gamma = y0 norm[10] + norm[12], H = y1 norm[11] + norm[13] (flux closure),
 * or m_D = y0 norm[10] + norm[12], m_eps = y1 norm[11] + norm[13], each
 * clamped to [1/4, 4] (multiplier closure: eqs. (12)-(13) with D_e, its
 * slope and the diffusion term of eq. (17) at the face times m_D, and mu_eps,
 * D_eps and the slope of D_eps times m_eps; the multipliers of a step are the
 * network's answer to the previous step's face inputs, 1 on the first step
 * after pc_fluid_set_state or a closure change).
 * All calls are asynchronous on the stream given at init unless noted.
 */
#ifndef PC_FLUID_H
#define PC_FLUID_H

#include "pc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pc_fluid_column {
    double L;       /* column length [m] */
    double Ngas;    /* gas density [m^-3] */
    double E0;      /* imposed mean field [V/m] */
    double nu_w;    /* radial loss frequency [1/s] (eq. (2)) */
    double muiN;    /* ion mobility x N [1/(V m s)] */
} pc_fluid_column;

typedef struct pc_fluid_config {
    int32_t n_columns, n_cells, table_len, pad;
    double dt, T_min, T_step, n_floor;
} pc_fluid_config;

typedef struct pc_fluid* pc_fluid_handle;

/* Workspace bytes (validates the config). */
pc_status pc_fluid_query(const pc_fluid_config* cfg, int64_t* workspace_bytes);
/* Create: cols (host, n_columns entries) and table (host double
 * [table_len][6]) are copied into the workspace (blocking). */
pc_status pc_fluid_init(const pc_fluid_config* cfg, const pc_fluid_column* cols, const double* table,
                        void* workspace, size_t bytes, void* hip_stream, pc_fluid_handle* out);
pc_status pc_fluid_set_state(pc_fluid_handle h, const float* n, const float* w);
/* (either pointer may be null) */
pc_status pc_fluid_get_state(pc_fluid_handle h, float* n, float* w);
/* Closure: mlp_packed = null selects eqs. (12)-(13) with the table;
 * otherwise the packed network of pc_mlp_pack with norm (host float[14]). */
pc_status pc_fluid_set_closure(pc_fluid_handle h, const void* mlp_packed, const float* norm);
/* Multiplier closure (the fluxes stay those of eqs. (12)-(13), so the
 * implicit diffusion split keeps its sign whatever the network answers):
 * mlp_packed and norm as above, both required. */
pc_status pc_fluid_set_closure_multipliers(pc_fluid_handle h, const void* mlp_packed, const float* norm);
pc_status pc_fluid_step(pc_fluid_handle h, int64_t n_steps);
/* Face values of the last step: flux, energy flux (table and multiplier
 * closures only) and field at face j (between cells j and j+1); any pointer
 * may be null. */
pc_status pc_fluid_get_faces(pc_fluid_handle h, float* gamma, float* H, float* E);
/* Batched cyclic tridiagonal solve a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j
 * (indices mod n, n a power of two <= 4096; device double [n_systems][n]);
 * the solution overwrites d.  Cyclic reduction, one workgroup per system. */
pc_status pc_cyclic_tridiag(const double* a, const double* b, const double* c, double* d,
                            int32_t n_systems, int32_t n, void* hip_stream);
void pc_fluid_destroy(pc_fluid_handle h);
const char* pc_fluid_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
