// device.h -- shared device-side definitions of the gfx950 PIC-MCC kernels.
//
// Column parameters, the counter-based random stream, isotropic directions,
// Maxwellian draws and the synthetic cross sections.  Every floating-point
// expression here is written in a fixed operation order and compiled without
// FMA contraction (-ffp-contract=off) so that results do not depend on the
// compiler's scheduling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcdev {

constexpr int kElectron = 0;
constexpr int kIon = 1;

// Philox stream tags (fourth counter word)
constexpr uint32_t kStreamElectronStep = 0;
constexpr uint32_t kStreamIonStep = 1;
constexpr uint32_t kStreamElectronLoad = 2;
constexpr uint32_t kStreamIonLoad = 3;
constexpr uint32_t kStreamVictimE = 4;   // pair sink: electron victims (counter word 0: rank)
constexpr uint32_t kStreamVictimI = 5;   // pair sink: ion victims
constexpr uint32_t kStreamEmit = 6;      // cathode emission (counter word 0: the new id)

// event codes (same values as the public header)
constexpr uint8_t kEvNone = 0, kEvElastic = 1, kEvExcite = 2, kEvIonize = 3, kEvWall = 4,
                  kEvAbsorb = 5, kEvCX = 6, kEvNull = 7;

// device error bits
constexpr uint32_t kErrECap = 1u, kErrGCap = 2u, kErrNuMax = 4u, kErrIds = 8u, kErrRange = 16u,
                   kErrBirths = 32u, kErrLosses = 64u, kErrCapacity = 128u, kErrField = 256u;

// charge of one macroparticle in fixed point: 25 fractional bits, so that the
// weights of 64 lanes (each <= 2^25) sum below 2^32
constexpr int64_t kUnit = int64_t(1) << 25;
constexpr double kUnitD = 33554432.0;

struct Counters {
    int64_t n[2];        // live particles
    int64_t next_id[2];  // next id per species
    int64_t step;        // index of the step being / to be executed
    uint32_t err;        // sticky error bits
    uint32_t pad0;
    int64_t nb;          // ionizations recorded in the current step
    int64_t nh[2];       // losses recorded in the current step
    int64_t births_last;       // balanced sink: ionizations of the previous step
    int64_t births_since_ion;  // balanced sink: ionizations since the last ion step
    // bounded column with an external circuit and cathode emission (section V)
    double V;            // anode potential of the next field solve [V]
    double J;            // conduction current density of the last step [A/m^2]
    int64_t field_loaded; // finish: step index + 1 once the field half holds that step's charges
    int64_t pad2;
    int64_t vsum_i;      // ions' sum of v_x (2^-20 m/s units) of the last ion step (held)
    double carry;        // fractional emitted electrons carried to the next step
    int64_t pad1[2];
};

struct Birth {           // one ionization event (56 bytes)
    uint32_t pid;        // id of the ionizing electron
    uint32_t slot;       // its array slot during the step
    double x;            // position
    double eps;          // energy before the collision [eV]
    double vs[3];        // scratch: scattered velocity (large-step fallback)
    double pad;
};

// One particle buffer (FP64): x and vx are read and written by every push, the
// transverse velocity (vy, vz) only by the few collision candidates of a step,
// so the pair is interleaved: a candidate touches one 16-byte element (one
// cache line) instead of two lines of two arrays.
struct Soa {
    double* x;
    double* vx;
    double2* vt;         // (vy, vz)
    uint32_t* id;
};

// FP32 particle buffer: cell-relative position (cell index, offset in [0,1))
// and velocities in cells per step of the species (electron: dt, ion: S dt)
struct Soa32 {
    int32_t* cell;
    float* off;
    float* vx;
    float2* vt;          // (vy, vz)
    uint32_t* id;
};

// Caller-side FP64 arrays (state exchange through the C ABI): separate
// vy and vz; any pointer may be null where documented.
struct SoaIO {
    double* x;
    double* vx;
    double* vy;
    double* vz;
    uint32_t* id;
};

struct Params {
    // grid
    int32_t nc, nn, periodic, ion_subcycle;
    double L, dx, inv_dx;
    // time stepping and species
    double dt, dti, qmdt_e, qmdt_i, c_eps, sig_a;
    // collisions
    double Ng, nu_max, P_null, T_we, T_wi, P_cx, g_cap, eps_cap, mr2;
    double el_A, el_B, ex_U, sx4, iz_U, si4, opb_w;
    int32_t el_pos, share_equal, poisson, pad0;
    // field
    double fpc, E0, V;
    uint32_t key0, key1;
    // integer forms of the per-step thresholds on the 52-bit draw k = r >> 12
    // (k < T is the same decision as (k + 1/2) 2^-52 < P for T = ceil(P 2^52 - 1/2))
    uint64_t kn_e, kw_e, kw_i, kcx;   // kw_*: fixed sink; the balanced sink derives them per step
    int32_t balanced, pair;         // pair: one electron and one ion removed per ionization
    uint32_t* slot_of[2];           // pair sink: slot of each id (ids dense in [0, next_id))
    // bounded column, section V: cathode emission and a series resistor
    int32_t emit, circuit;
    double emit_n;                  // emitted electrons per step, J_e0 dt / (e W)
    double emit_sig;                // sqrt(e T_c / m_e): thermal speed of emitted electrons
    double circ_R;                  // series resistance [ohm m^2]
    double circ_a;                  // R eps0 / (L dt)
    double circ_jf;                 // e W / L per 2^-20 m/s: current density of one velocity unit
    int64_t* csum;                  // v_x sums of the step: 64 electron slots, 64 ion slots
    // FP32 path: velocity scales (m/s per cell/step) and field scales
    double u2v_e, u2v_i;            // dx/dt, dx/dt_i
    double efs_e, efs_i;            // q dt^2/(m dx), q dt_i^2/(M dx)
    float* Ef_e;                    // E scaled to cells/step^2, n_nodes + 1 (ghost)
    float* Ef_i;
    int64_t cap, max_births, max_holes;
    Counters* cnt;
    Birth* births;
    uint32_t* holes[2];
    uint32_t* cand;      // electron collision candidates (slot indices): each block of
                         // the push kernel lists its own from the start of its chunk
    uint2* cand_w;       // their Philox block-0 words 2, 3 (the process draw u1)
    uint32_t* lists;     // compaction scratch: 2 * max_holes entries
    uint32_t* bitmap;    // compaction scratch: max_holes bits
    int64_t* iz;         // ionizations per cell
    double* E;           // n_nodes + 1 (periodic ghost E[nc] = E[0])
    int32_t* sort_cnt;   // counting-sort histogram, n_cells
    int32_t* sort_off;   // counting-sort cursors, n_cells
};

// One column of a batch: its parameters and both buffers of each particle
// store and charge array (device table read by the batched kernels).
struct ColumnDev {
    Params P;
    Soa soa[2][2];       // [species][buffer], FP64 columns
    Soa32 soa32[2][2];   // [species][buffer], FP32 columns
    int64_t* rho[2][2];  // [species][buffer]
};

// chunk k of nk of one column's particle array
struct BatchItem {
    int32_t col, k, nk, pad;
};

// buffer indices of one batched step (shared by every column of the batch)
struct BatchStep {
    int32_t cur[2];      // particle buffer per species
    int32_t re_new;      // electron charge buffer receiving this step's deposit
    int32_t re_old;      // electron charge buffer cleared for the next step
    int32_t ri_use;      // ion charge buffer used by the field (deposited on ion steps)
    int32_t ri_old;      // ion charge buffer cleared on ion steps, else -1
    int32_t ion;         // ions advance on this step
    int32_t pad;
};


// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): per round two 32x32->64
// products of counter words 0 and 2 with the round multipliers, the high
// halves XORed into words 1 and 3 and the key; key += Weyl constants.
struct U4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p = uint64_t(0xD2511F53u) * c0;
        const uint64_t q = uint64_t(0xCD9E8D57u) * c2;
        const uint32_t n0 = uint32_t(q >> 32) ^ c1 ^ k0;
        const uint32_t n2 = uint32_t(p >> 32) ^ c3 ^ k1;
        c1 = uint32_t(q);
        c3 = uint32_t(p);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// open-interval uniforms: 52 bits from a word pair, or one 32-bit word
__device__ __forceinline__ double unif52(uint32_t lo, uint32_t hi)
{
    const uint64_t r = (uint64_t(hi) << 32) | lo;
    return (double(r >> 12) + 0.5) * 0x1p-52;
}
__device__ __forceinline__ double unif32(uint32_t w) { return (double(w) + 0.5) * 0x1p-32; }

// Sequential words from Philox blocks 1, 2, 3, ... of (id, step, stream).
struct WordStream {
    uint32_t id, step, stream, k0, k1, block;
    U4 buf;
    int pos;
    __device__ WordStream(uint32_t id_, uint32_t step_, uint32_t stream_, uint32_t k0_, uint32_t k1_)
        : id(id_), step(step_), stream(stream_), k0(k0_), k1(k1_), block(0), buf{0, 0, 0, 0}, pos(4) {}
    __device__ __forceinline__ uint32_t next()
    {
        if (pos == 4) {
            block += 1;
            buf = philox10(id, step, block, stream, k0, k1);
            pos = 0;
        }
        const uint32_t w = pos == 0 ? buf.a : pos == 1 ? buf.b : pos == 2 ? buf.c : buf.d;
        ++pos;
        return w;
    }
    __device__ __forceinline__ double u() { return unif32(next()); }
};

// isotropic unit vector: Marsaglia (1972) point in the unit disk, at most 64
// tries, then the +z pole
__device__ __forceinline__ void isotropic(WordStream& ws, double& nx, double& ny, double& nz)
{
    for (int t = 0; t < 64; ++t) {
        const double a = 2.0 * ws.u() - 1.0;
        const double b = 2.0 * ws.u() - 1.0;
        const double s = a * a + b * b;
        if (s < 1.0) {
            const double r = 2.0 * sqrt(1.0 - s);
            nx = a * r;
            ny = b * r;
            nz = 1.0 - 2.0 * s;
            return;
        }
    }
    nx = 0.0;
    ny = 0.0;
    nz = 1.0;
}

// two standard normals by the Marsaglia-Bray polar method, at most 64 tries
__device__ __forceinline__ void normal_pair(WordStream& ws, double& g0, double& g1)
{
    for (int t = 0; t < 64; ++t) {
        const double a = 2.0 * ws.u() - 1.0;
        const double b = 2.0 * ws.u() - 1.0;
        const double s = a * a + b * b;
        if (s < 1.0 && s > 0.0) {
            const double f = sqrt(-2.0 * log(s) / s);
            g0 = a * f;
            g1 = b * f;
            return;
        }
    }
    g0 = 0.0;
    g1 = 0.0;
}

// three normals: a full pair, then the first of a second pair
__device__ __forceinline__ void normal3(WordStream& ws, double& g0, double& g1, double& g2)
{
    double h;
    normal_pair(ws, g0, g1);
    normal_pair(ws, g2, h);
}

// ---------------------------------------------------------- cross sections
__device__ __forceinline__ double sigma_elastic(const Params& P, double eps)
{
    if (P.el_pos) return P.el_A + P.el_B * sqrt(eps);
    return eps > 0.0 ? P.el_A + P.el_B / sqrt(eps) : P.el_A;
}
// Thomson-like lumped inelastic channel: 4 smax (U/eps)(1 - U/eps), eps > U
__device__ __forceinline__ double sigma_inelastic(double eps, double U, double s4)
{
    if (eps > U) {
        const double t = U / eps;
        return s4 * t * (1.0 - t);
    }
    return 0.0;
}

// cell index and fraction of a position in [0, L)
__device__ __forceinline__ int cell_frac(const Params& P, double x, double& f)
{
    const double s = x * P.inv_dx;
    int j = int(s);
    if (j > P.nc - 1) j = P.nc - 1;
    if (j < 0) j = 0;   // never taken for x in [0, L); keeps reads in bounds
    f = s - double(j);
    return j;
}

// 25-bit weight of a cell fraction f in [0, 1]: trunc(f 2^25), at most 2^25.
// f 2^25 < 2^32, so the unsigned 32-bit conversion truncates exactly as a
// 64-bit one would, in one instruction.
__device__ __forceinline__ int64_t frac_units(double f)
{
    const uint32_t a = uint32_t(f * kUnitD);
    return int64_t(a > uint32_t(kUnit) ? uint32_t(kUnit) : a);
}

// Integer threshold T on the 52-bit draw k with k < T  <=>  (k + 1/2) 2^-52 < p
// (the same double arithmetic as the host's).
__device__ __forceinline__ uint64_t thr52(double p)
{
    if (!(p > 0.0)) return 0;
    if (!(p < 1.0)) return uint64_t(1) << 52;
    return uint64_t(ceil(p * 4503599627370496.0 - 0.5));
}

// Sink thresholds of the current step.  Balanced sink (the paper removes an
// electron-ion pair per ionization to keep the particle number constant):
// survival 1 - (ionizations since the species' previous step) / (its count).
__device__ __forceinline__ uint64_t sink_threshold(const Params& P, int species)
{
    if (!P.balanced) return species == 0 ? P.kw_e : P.kw_i;
    const int64_t n = P.cnt->n[species];
    const int64_t b = species == 0 ? P.cnt->births_last : P.cnt->births_since_ion;
    return n > 0 ? thr52(1.0 - double(b) / double(n)) : (uint64_t(1) << 52);
}

}  // namespace pcdev
