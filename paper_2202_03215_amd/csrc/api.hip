// api.hip -- host implementation of the C ABI declared in include/pc.h.
//
// The handle owns host metadata only; every device byte lives in the
// caller's workspace.  Derived constants follow the model of section II of
// the paper (Boeuf): gas density from p and T_g, leapfrog charge-to-mass
// factors, the null-collision bound over [0, eps_cap], the per-step removal
// probability of the radial sink (eq. (2) frequency), the Gauss's-law field
// jump per fixed-point charge unit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pc.h"
#include "device.h"
#include "launch.h"

using pcdev::Counters;
using pcdev::Params;
using pcdev::Soa;
using pcdev::Soa32;

namespace {

// CODATA 2018
constexpr double kQe = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kKb = 1.380649e-23;
constexpr double kEps0 = 8.8541878128e-12;
const double kTorr = 101325.0 / 760.0;

thread_local std::string g_last_error;

pc_status fail(pc_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

pc_status hip_fail(hipError_t e, const char* where)
{
    return fail(PC_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

// Integer threshold T on the 52-bit draw k with k < T  <=>  (k + 1/2) 2^-52 < p
// (p 2^52 - 1/2 is exact in double for p < 1).
uint64_t thr52(double p)
{
    if (!(p > 0.0)) return 0;
    if (!(p < 1.0)) return uint64_t(1) << 52;
    return uint64_t(std::ceil(p * 4503599627370496.0 - 0.5));
}

struct Derived {
    int nc, nn, periodic, fp32, pair;
    double dx, inv_dx, dti, Ng, M, c_eps, qmdt_e, qmdt_i, W, fpc, E0;
    double sig_a, sig_e0, sig_i0, mr2, sx4, si4;
    double nu_max, P_null, T_we, T_wi, P_cx;
    int64_t n0, cap, max_births, max_holes;
};

double sig_el_host(const pc_config& c, double eps)
{
    if (c.el_p > 0.0) return c.el_A + c.el_B * std::sqrt(eps);
    return eps > 0.0 ? c.el_A + c.el_B / std::sqrt(eps) : c.el_A;
}

double sig_in_host(double eps, double U, double s4)
{
    if (eps > U) {
        const double t = U / eps;
        return s4 * t * (1.0 - t);
    }
    return 0.0;
}

pc_status derive(const pc_config* c, Derived* d)
{
    if (!c || !d) return fail(PC_ERR_INVALID_ARG, "null config");
    if (c->bc != PC_BOUNDED && c->bc != PC_PERIODIC) return fail(PC_ERR_INVALID_ARG, "bc");
    if (c->n_cells < 2) return fail(PC_ERR_INVALID_ARG, "n_cells < 2");
    if (!(c->L > 0.0) || !(c->dt > 0.0) || c->ppc < 1 || c->ion_subcycle < 1)
        return fail(PC_ERR_INVALID_ARG, "L, dt, ppc and ion_subcycle must be positive");
    if (c->el_p != 0.5 && c->el_p != -0.5) return fail(PC_ERR_INVALID_ARG, "el_p must be +0.5 or -0.5");
    if (c->wall_mode != PC_WALL_OFF && c->wall_mode != PC_WALL_FIXED && c->wall_mode != PC_WALL_BALANCED &&
        c->wall_mode != PC_WALL_PAIR)
        return fail(PC_ERR_INVALID_ARG, "wall_mode");
    // the pair sink keeps ids dense, which electrode absorption would break
    if (c->wall_mode == PC_WALL_PAIR && c->bc != PC_PERIODIC)
        return fail(PC_ERR_INVALID_ARG, "the pair sink needs a periodic column");
    if (!(c->emit_J >= 0.0) || !(c->circuit_R >= 0.0) || (c->emit_J > 0.0 && !(c->emit_T > 0.0)))
        return fail(PC_ERR_INVALID_ARG, "emit_J and circuit_R must be >= 0, emit_T > 0 with emission");
    if ((c->emit_J > 0.0 || c->circuit_R > 0.0) && c->bc != PC_BOUNDED)
        return fail(PC_ERR_INVALID_ARG, "cathode emission and the external circuit need a bounded column");
    if (c->energy_sharing != PC_SHARE_OPB && c->energy_sharing != PC_SHARE_EQUAL)
        return fail(PC_ERR_INVALID_ARG, "energy_sharing");
    if (!(c->eps_cap > 0.0) || !(c->g_cap > 0.0) || !(c->M_amu > 0.0) || !(c->n0 > 0.0) || !(c->Tg > 0.0))
        return fail(PC_ERR_INVALID_ARG, "eps_cap, g_cap, M_amu, n0, Tg must be positive");
    if (c->sort_interval < 0) return fail(PC_ERR_INVALID_ARG, "sort_interval < 0");
    if (c->launch_blocks < 0 || c->launch_blocks > 65536) return fail(PC_ERR_INVALID_ARG, "launch_blocks");
    if (c->precision != PC_FP64 && c->precision != PC_FP32) return fail(PC_ERR_INVALID_ARG, "precision");
    d->nc = c->n_cells;
    d->periodic = c->bc == PC_PERIODIC;
    d->fp32 = c->precision == PC_FP32;
    d->pair = c->wall_mode == PC_WALL_PAIR;
    d->nn = d->periodic ? d->nc : d->nc + 1;
    if (d->nn > pclaunch::max_nodes()) return fail(PC_ERR_INVALID_ARG, "too many nodes for the field solve");
    d->dx = c->L / double(d->nc);
    d->inv_dx = double(d->nc) / c->L;
    d->dti = double(c->ion_subcycle) * c->dt;
    d->Ng = c->p_torr * kTorr / (kKb * c->Tg);
    d->M = c->M_amu * kAmu;
    d->c_eps = 0.5 * kMe / kQe;
    d->qmdt_e = (-kQe * c->dt) / kMe;
    d->qmdt_i = (kQe * d->dti) / d->M;
    d->W = c->n0 * d->dx / double(c->ppc);
    d->fpc = kQe * d->W / pcdev::kUnitD / kEps0;
    d->E0 = c->V / c->L;
    d->sig_a = std::sqrt(kKb * c->Tg / d->M);
    d->sig_e0 = std::sqrt(c->Te0_eV * kQe / kMe);
    d->sig_i0 = std::sqrt(kKb * c->Ti0_K / d->M);
    d->mr2 = 2.0 * kMe / d->M;
    d->sx4 = 4.0 * c->ex_smax;
    d->si4 = 4.0 * c->iz_smax;
    // null-collision bound: largest Ng sigma_tot v on a 65536-interval grid of
    // [0, eps_cap], with a 0.1 % margin
    {
        const int G = 65536;
        double mx = 0.0;
        for (int k = 0; k <= G; ++k) {
            const double eps = c->eps_cap * double(k) / double(G);
            const double v = std::sqrt(eps / d->c_eps);
            const double s = sig_el_host(*c, eps) + sig_in_host(eps, c->ex_U, d->sx4) +
                             sig_in_host(eps, c->iz_U, d->si4);
            const double nu = s * v * d->Ng;
            if (nu > mx) mx = nu;
        }
        d->nu_max = mx * 1.001;
    }
    d->P_null = 1.0 - std::exp(-d->nu_max * c->dt);
    if (c->wall_mode == PC_WALL_FIXED) {
        d->T_we = std::exp(-c->nu_w * c->dt);
        d->T_wi = std::exp(-c->nu_w * d->dti);
    } else {
        d->T_we = 2.0;
        d->T_wi = 2.0;
    }
    d->P_cx = 1.0 - std::exp(-d->Ng * c->cx_sigma * c->g_cap * d->dti);
    // stability (section II): dt < 0.2 / w_pe and dx < lambda_De; collision
    // probabilities per step small enough for one collision per step
    const double wpe = std::sqrt(c->n0 * kQe * kQe / (kEps0 * kMe));
    if (!(c->dt < 0.2 / wpe))
        return fail(PC_ERR_UNSTABLE_CONFIG, "dt must be below 0.2/w_pe");
    if (c->Te0_eV > 0.0) {
        const double lde = std::sqrt(kEps0 * c->Te0_eV / (c->n0 * kQe));
        if (!(d->dx < lde)) return fail(PC_ERR_UNSTABLE_CONFIG, "dx must be below the Debye length");
    }
    if (!(d->nu_max * c->dt <= 0.1)) return fail(PC_ERR_UNSTABLE_CONFIG, "nu_max dt above 0.1");
    if (!(d->Ng * c->cx_sigma * c->g_cap * d->dti <= 0.1))
        return fail(PC_ERR_UNSTABLE_CONFIG, "ion null-collision probability above 0.1");
    d->n0 = int64_t(c->ppc) * d->nc;
    const double capf = c->capacity > 1.0 ? c->capacity : 1.0;
    int64_t cap = int64_t(std::ceil(double(d->n0) * capf));
    cap = std::max<int64_t>(1024, (cap + 255) & ~int64_t(255));
    // particle arrays are addressed with 32-bit byte offsets (8-byte fields)
    if (cap > (int64_t(1) << 29)) return fail(PC_ERR_INVALID_ARG, "capacity above 2^29 particles");
    d->cap = cap;
    d->max_births = std::max<int64_t>(4096, cap / 256);
    d->max_holes = std::max<int64_t>(8192, cap / 64);
    return PC_OK;
}

struct Layout {
    int64_t counters, soa[2][2][6], rho[2][2], E, Ef_e, Ef_i, births, holes[2], cand, cand_w, lists, bitmap, iz,
        sort_cnt, sort_off, slot_of[2], csum, total;
};

Layout layout(const Derived& d)
{
    Layout L{};
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.counters = take(sizeof(Counters));
    // FP64: x, vx (8 B), (vy, vz) (16 B), id (4 B); FP32: cell, offset, vx (4 B), (vy, vz) (8 B), id
    for (int s = 0; s < 2; ++s)
        for (int b = 0; b < 2; ++b) {
            const int64_t w = d.fp32 ? 4 : 8;
            L.soa[s][b][0] = take(d.cap * w);
            L.soa[s][b][1] = take(d.cap * w);
            L.soa[s][b][2] = take(d.cap * 2 * w);
            L.soa[s][b][3] = take(d.cap * 4);
            if (d.fp32) L.soa[s][b][4] = take(d.cap * 4);
        }
    for (int s = 0; s < 2; ++s)
        for (int b = 0; b < 2; ++b) L.rho[s][b] = take(int64_t(d.nn) * 8);
    L.E = take(int64_t(d.nn + 1) * 8);
    L.Ef_e = d.fp32 ? take(int64_t(d.nn + 1) * 4) : -1;
    L.Ef_i = d.fp32 ? take(int64_t(d.nn + 1) * 4) : -1;
    L.births = take(d.max_births * int64_t(sizeof(pcdev::Birth)));
    L.holes[0] = take(d.max_holes * 4);
    L.holes[1] = take(d.max_holes * 4);
    L.cand = take(d.cap * 4);
    L.cand_w = take(d.cap * 8);
    L.lists = take(2 * d.max_holes * 4);
    L.bitmap = take((d.max_holes / 32 + 1) * 4);
    L.iz = take(int64_t(d.nc) * 8);
    L.sort_cnt = take(int64_t(d.nc) * 4);
    L.sort_off = take(int64_t(d.nc) * 4);
    L.slot_of[0] = d.pair ? take(d.cap * 4) : -1;
    L.slot_of[1] = d.pair ? take(d.cap * 4) : -1;
    L.csum = take(128 * 8);
    L.total = o;
    return L;
}

}  // namespace

struct pc_column {
    pc_config cfg;
    Derived d;
    Params P;
    hipStream_t st;
    Soa buf[2][2];       // FP64 stores
    Soa32 buf32[2][2];   // FP32 stores
    int fp32;
    int cur[2];
    int64_t* rho[2][2];
    int re_cur, ri_cur;
    int64_t step;
    int poisoned;
    uint8_t* ev[2];
    int64_t evlen[2];
    int grid;     // blocks of the streaming particle kernels
    Counters host_cnt;
    std::vector<hipEvent_t> tev;   // timer pool: 2 events per launch
    int64_t tcount;
    int use_graphs;                // replay captured HIP graphs of whole steps
    struct Graph {
        int64_t key[6];            // step % period, charge and particle buffer parities, length
        hipGraphExec_t exec;
        int64_t used;              // last use (eviction order)
    };
    std::vector<Graph> graphs;     // whole periods and shorter remainders, at most kMaxGraphs
    int64_t graph_clock;
    int batch_member;              // owned and stepped by a batch
    int slots_dirty;               // pair sink: the id -> slot map is rebuilt before the next step
};

namespace {

pc_status map_errors(uint32_t e)
{
    if (e == 0) return PC_OK;
    if (e & (pcdev::kErrRange | pcdev::kErrField)) return fail(PC_ERR_NONFINITE, "position or field out of range");
    if (e & (pcdev::kErrBirths | pcdev::kErrLosses | pcdev::kErrCapacity))
        return fail(PC_ERR_CAPACITY, "birth, loss or particle capacity exceeded");
    if (e & (pcdev::kErrECap | pcdev::kErrNuMax)) return fail(PC_ERR_ECAP, "electron energy above eps_cap");
    if (e & pcdev::kErrGCap) return fail(PC_ERR_GCAP, "ion-atom relative speed above g_cap");
    if (e & pcdev::kErrIds) return fail(PC_ERR_IDS, "id space exhausted");
    return fail(PC_ERR_HIP, "unknown device error");
}

pc_status read_counters(pc_column* h)
{
    HIPCHK(hipMemcpyAsync(&h->host_cnt, h->P.cnt, sizeof(Counters), hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return PC_OK;
}

pc_status write_counters(pc_column* h)
{
    HIPCHK(hipMemcpyAsync(h->P.cnt, &h->host_cnt, sizeof(Counters), hipMemcpyHostToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return PC_OK;
}

Soa soa_of(const pc_column* h, int s) { return h->buf[s][h->cur[s]]; }

// Ions are advanced once per subcycle and move far less per step than
// electrons, so their array order decays more slowly: they are sorted at
// every kIonSortEvery-th sort (measured on the 400k + 400k column with K = 20:
// 26.47 us per step against 26.93 sorting both species every time; every 4th
// or 8th sort gains less, the longer graph period costing more).  The order
// of the arrays changes no result.
constexpr int kIonSortEvery = 2;

pc_status run_sort(pc_column* h, bool ions, bool launch = true)
{
    for (int s = 0; s < (ions ? 2 : 1); ++s) {
        if (launch) {
            if (h->fp32)
                HIPCHK(pclaunch::sort(h->P, s, h->buf32[s][h->cur[s]], h->buf32[s][1 - h->cur[s]], h->grid, h->st));
            else
                HIPCHK(pclaunch::sort(h->P, s, h->buf[s][h->cur[s]], h->buf[s][1 - h->cur[s]], h->grid, h->st));
        }
        h->cur[s] = 1 - h->cur[s];
    }
    return PC_OK;
}

}  // namespace

extern "C" {

pc_status pc_query_sizes(const pc_config* cfg, pc_sizes* out)
{
    if (!out) return fail(PC_ERR_INVALID_ARG, "null output");
    Derived d;
    const pc_status s = derive(cfg, &d);
    if (s != PC_OK) return s;
    const Layout L = layout(d);
    out->workspace_bytes = L.total;
    out->capacity = d.cap;
    out->max_births = d.max_births;
    out->max_losses = d.max_holes;
    out->n_nodes = d.nn;
    out->n_cells = d.nc;
    out->nu_max = d.nu_max;
    out->p_null = d.P_null;
    out->p_cx = d.P_cx;
    return PC_OK;
}

}  // extern "C"

// Set up one column in device memory at `base` (layout(d).total bytes, 256-byte
// aligned): particle loads, first deposit and field, leapfrog half step.
static pc_status column_init(const pc_config* cfg, const Derived& d, char* base, hipStream_t stream,
                             pc_column** out)
{
    pc_status s = PC_OK;
    const Layout L = layout(d);
    pc_column* h = new (std::nothrow) pc_column();
    if (!h) return fail(PC_ERR_INVALID_ARG, "host allocation failed");
    h->cfg = *cfg;
    h->d = d;
    h->st = stream;
    h->fp32 = d.fp32;
    for (int sp = 0; sp < 2; ++sp)
        for (int b = 0; b < 2; ++b) {
            if (d.fp32) {
                Soa32& q = h->buf32[sp][b];
                q.cell = reinterpret_cast<int32_t*>(base + L.soa[sp][b][0]);
                q.off = reinterpret_cast<float*>(base + L.soa[sp][b][1]);
                q.vt = reinterpret_cast<float2*>(base + L.soa[sp][b][2]);
                q.id = reinterpret_cast<uint32_t*>(base + L.soa[sp][b][3]);
                q.vx = reinterpret_cast<float*>(base + L.soa[sp][b][4]);
            } else {
                Soa& q = h->buf[sp][b];
                q.x = reinterpret_cast<double*>(base + L.soa[sp][b][0]);
                q.vx = reinterpret_cast<double*>(base + L.soa[sp][b][1]);
                q.vt = reinterpret_cast<double2*>(base + L.soa[sp][b][2]);
                q.id = reinterpret_cast<uint32_t*>(base + L.soa[sp][b][3]);
            }
            h->rho[sp][b] = reinterpret_cast<int64_t*>(base + L.rho[sp][b]);
        }
    Params& P = h->P;
    P.nc = d.nc;
    P.nn = d.nn;
    P.periodic = d.periodic;
    P.ion_subcycle = cfg->ion_subcycle;
    P.L = cfg->L;
    P.dx = d.dx;
    P.inv_dx = d.inv_dx;
    P.dt = cfg->dt;
    P.dti = d.dti;
    P.qmdt_e = d.qmdt_e;
    P.qmdt_i = d.qmdt_i;
    P.c_eps = d.c_eps;
    P.sig_a = d.sig_a;
    P.Ng = d.Ng;
    P.nu_max = d.nu_max;
    P.P_null = d.P_null;
    P.T_we = d.T_we;
    P.T_wi = d.T_wi;
    P.P_cx = d.P_cx;
    P.g_cap = cfg->g_cap;
    P.eps_cap = cfg->eps_cap;
    P.mr2 = d.mr2;
    P.el_A = cfg->el_A;
    P.el_B = cfg->el_B;
    P.ex_U = cfg->ex_U;
    P.sx4 = d.sx4;
    P.iz_U = cfg->iz_U;
    P.si4 = d.si4;
    P.opb_w = cfg->opb_w;
    P.el_pos = cfg->el_p > 0.0;
    P.share_equal = cfg->energy_sharing == PC_SHARE_EQUAL;
    P.poisson = cfg->poisson != 0;
    P.fpc = d.fpc;
    P.E0 = d.E0;
    P.V = cfg->V;
    P.key0 = uint32_t(cfg->seed);
    P.key1 = uint32_t(cfg->seed >> 32);
    P.kn_e = thr52(d.P_null);
    P.kw_e = thr52(d.T_we);
    P.kw_i = thr52(d.T_wi);
    P.kcx = thr52(d.P_cx);
    P.balanced = cfg->wall_mode == PC_WALL_BALANCED;
    P.pair = d.pair;
    P.emit = cfg->emit_J > 0.0;
    P.circuit = cfg->circuit_R > 0.0;
    P.emit_n = cfg->emit_J * cfg->dt / (kQe * d.W);
    P.emit_sig = std::sqrt(kQe * cfg->emit_T / kMe);
    P.circ_R = cfg->circuit_R;
    P.circ_a = cfg->circuit_R * kEps0 / (cfg->L * cfg->dt);
    P.circ_jf = kQe * d.W / cfg->L / 1048576.0;
    P.csum = reinterpret_cast<int64_t*>(base + L.csum);
    P.slot_of[0] = d.pair ? reinterpret_cast<uint32_t*>(base + L.slot_of[0]) : nullptr;
    P.slot_of[1] = d.pair ? reinterpret_cast<uint32_t*>(base + L.slot_of[1]) : nullptr;
    P.u2v_e = d.dx / cfg->dt;
    P.u2v_i = d.dx / d.dti;
    P.efs_e = (-kQe * cfg->dt * cfg->dt) / (kMe * d.dx);
    P.efs_i = (kQe * d.dti * d.dti) / (d.M * d.dx);
    P.Ef_e = d.fp32 ? reinterpret_cast<float*>(base + L.Ef_e) : nullptr;
    P.Ef_i = d.fp32 ? reinterpret_cast<float*>(base + L.Ef_i) : nullptr;
    P.cap = d.cap;
    P.max_births = d.max_births;
    P.max_holes = d.max_holes;
    P.cnt = reinterpret_cast<Counters*>(base + L.counters);
    P.births = reinterpret_cast<pcdev::Birth*>(base + L.births);
    P.holes[0] = reinterpret_cast<uint32_t*>(base + L.holes[0]);
    P.holes[1] = reinterpret_cast<uint32_t*>(base + L.holes[1]);
    P.cand = reinterpret_cast<uint32_t*>(base + L.cand);
    P.cand_w = reinterpret_cast<uint2*>(base + L.cand_w);
    P.lists = reinterpret_cast<uint32_t*>(base + L.lists);
    P.bitmap = reinterpret_cast<uint32_t*>(base + L.bitmap);
    P.iz = reinterpret_cast<int64_t*>(base + L.iz);
    P.E = reinterpret_cast<double*>(base + L.E);
    P.sort_cnt = reinterpret_cast<int32_t*>(base + L.sort_cnt);
    P.sort_off = reinterpret_cast<int32_t*>(base + L.sort_off);
    // about one initial particle per thread of the advance kernels, with 1/32
    // headroom: a count a little above the initial one still gives every
    // block at most one 256-particle tile (the partition rounds chunks up to
    // multiples of 64, so 1563 blocks for 401k electrons make 320-particle
    // chunks, a second, nearly empty tile per block).  Measured on the 400k
    // column: 1563 blocks 26.46 us per step, 1600-1700 blocks 26.1, 3125
    // blocks 27.6, 4096 blocks 29.1.
    h->grid = cfg->launch_blocks > 0
                  ? cfg->launch_blocks
                  : int(std::min<int64_t>(4096, std::max<int64_t>(1, (d.n0 + d.n0 / 32 + 255) / 256)));
    h->cur[0] = h->cur[1] = 0;
    h->re_cur = h->ri_cur = 0;
    h->use_graphs = 1;
    h->graph_clock = 0;
    h->step = 0;

    auto cleanup = [&](pc_status st) {
        delete h;
        return st;
    };
    std::memset(&h->host_cnt, 0, sizeof(Counters));
    h->host_cnt.n[0] = h->host_cnt.n[1] = d.n0;
    h->host_cnt.next_id[0] = h->host_cnt.next_id[1] = d.n0;
    h->host_cnt.V = cfg->V;
    if ((s = write_counters(h)) != PC_OK) return cleanup(s);
    hipError_t e = hipSuccess;
    for (int sp = 0; sp < 2 && e == hipSuccess; ++sp)
        for (int b = 0; b < 2 && e == hipSuccess; ++b) e = pclaunch::fill_i64(h->rho[sp][b], d.nn, 0, h->st);
    if (e == hipSuccess) e = pclaunch::fill_i64(P.iz, d.nc, 0, h->st);
    if (e == hipSuccess) e = pclaunch::fill_i64(P.csum, 128, 0, h->st);
    if (e == hipSuccess) e = pclaunch::fill_i64(reinterpret_cast<int64_t*>(P.sort_cnt), (d.nc + 1) / 2, 0, h->st);
    if (d.fp32) {
        // FP32 columns: the loader draws in FP64 and converts each particle
        if (e == hipSuccess) e = pclaunch::load(P, 0, h->buf32[0][0], d.n0, d.sig_e0, h->st);
        if (e == hipSuccess) e = pclaunch::load(P, 1, h->buf32[1][0], d.n0, d.sig_i0, h->st);
    } else {
        if (e == hipSuccess) e = pclaunch::load(P, 0, h->buf[0][0], d.n0, d.sig_e0, h->st);
        if (e == hipSuccess) e = pclaunch::load(P, 1, h->buf[1][0], d.n0, d.sig_i0, h->st);
        if (e == hipSuccess) e = pclaunch::deposit(P, h->buf[0][0].x, d.n0, h->rho[0][0], h->st);
        if (e == hipSuccess) e = pclaunch::deposit(P, h->buf[1][0].x, d.n0, h->rho[1][0], h->st);
    }
    if (e != hipSuccess) return cleanup(hip_fail(e, "pc_init_column launch"));
    if (d.fp32) {
        e = pclaunch::deposit(P, h->buf32[0][0], d.n0, h->rho[0][0], h->st);
        if (e == hipSuccess) e = pclaunch::deposit(P, h->buf32[1][0], d.n0, h->rho[1][0], h->st);
    }
    if (e == hipSuccess) e = pclaunch::field(P, h->rho[0][0], h->rho[1][0], P.E, nullptr, 1, h->st);
    if (e == hipSuccess) e = pclaunch::scale_field(P, h->st);
    if (d.fp32) {
        if (e == hipSuccess) e = pclaunch::halfstep(P, h->buf32[0][0], 0, d.n0, h->st);
        if (e == hipSuccess) e = pclaunch::halfstep(P, h->buf32[1][0], 1, d.n0, h->st);
    } else {
        if (e == hipSuccess) e = pclaunch::halfstep(P, h->buf[0][0], d.n0, 0.5 * d.qmdt_e, h->st);
        if (e == hipSuccess) e = pclaunch::halfstep(P, h->buf[1][0], d.n0, 0.5 * d.qmdt_i, h->st);
    }
    if (e != hipSuccess) return cleanup(hip_fail(e, "pc_init_column launch"));
    if (cfg->sort_interval > 0 && (s = run_sort(h, true)) != PC_OK) return cleanup(s);
    if ((s = read_counters(h)) != PC_OK) return cleanup(s);
    if (h->host_cnt.err) return cleanup(map_errors(h->host_cnt.err));
    h->slots_dirty = d.pair;
    *out = h;
    return PC_OK;
}

extern "C" pc_status pc_init_column(const pc_config* cfg, void* workspace, size_t bytes, void* hip_stream,
                                    pc_handle* out)
{
    if (!out || !workspace) return fail(PC_ERR_INVALID_ARG, "null workspace or handle");
    *out = nullptr;
    Derived d;
    pc_status s = derive(cfg, &d);
    if (s != PC_OK) return s;
    const Layout L = layout(d);
    if (int64_t(bytes) < L.total) return fail(PC_ERR_WORKSPACE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) & 255u) return fail(PC_ERR_WORKSPACE, "workspace not 256-byte aligned");
    return column_init(cfg, d, static_cast<char*>(workspace), static_cast<hipStream_t>(hip_stream), out);
}

extern "C" {

// Enqueue one full time step on the column's stream and advance the host-side
// bookkeeping (step index, charge and sort buffer parities).  With time_it,
// the electron advance launch is bracketed by timer pair `slot`.  With
// launch false only the bookkeeping advances (the step is replayed from a
// graph).
static pc_status enqueue_step(pc_column* h, bool time_it, int64_t slot, bool launch = true)
{
    const int S = h->cfg.ion_subcycle;
    const int K = h->cfg.sort_interval;
    const bool ion = h->step % S == 0;
    if (!launch) {
        h->re_cur = 1 - h->re_cur;
        if (ion) h->ri_cur = 1 - h->ri_cur;
        h->step += 1;
        if (K > 0 && h->step % K == 0) return run_sort(h, h->step % (int64_t(K) * kIonSortEvery) == 0, false);
        return PC_OK;
    }
    int64_t* re_new = h->rho[0][1 - h->re_cur];
    int64_t* re_old = h->rho[0][h->re_cur];
    int64_t* ri_use = ion ? h->rho[1][1 - h->ri_cur] : h->rho[1][h->ri_cur];
    int64_t* ri_old = ion ? h->rho[1][h->ri_cur] : nullptr;
    hipEvent_t t0 = time_it ? h->tev[2 * slot] : nullptr, t1 = time_it ? h->tev[2 * slot + 1] : nullptr;
    if (h->fp32) {
        const Soa32 se = h->buf32[0][h->cur[0]], si = h->buf32[1][h->cur[1]];
        HIPCHK(pclaunch::advance(h->P, 0, se, re_new, h->ev[0], h->evlen[0], h->grid, h->st, t0, t1));
        if (ion) HIPCHK(pclaunch::advance(h->P, 1, si, ri_use, h->ev[1], h->evlen[1], h->grid, h->st));
        HIPCHK(pclaunch::finish(h->P, se, si, re_new, ri_use, re_old, ri_old, h->st));
    } else {
        const Soa se = soa_of(h, 0), si = soa_of(h, 1);
        HIPCHK(pclaunch::advance(h->P, 0, se, re_new, h->ev[0], h->evlen[0], h->grid, h->st, t0, t1));
        if (ion) HIPCHK(pclaunch::advance(h->P, 1, si, ri_use, h->ev[1], h->evlen[1], h->grid, h->st));
        HIPCHK(pclaunch::finish(h->P, se, si, re_new, ri_use, re_old, ri_old, h->st));
    }
    h->re_cur = 1 - h->re_cur;
    if (ion) h->ri_cur = 1 - h->ri_cur;
    h->step += 1;
    if (K > 0 && h->step % K == 0) return run_sort(h, h->step % (int64_t(K) * kIonSortEvery) == 0);
    return PC_OK;
}

static int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Steps after which every buffer parity returns: electron charge buffers
// alternate each step, ion charge buffers each ion step, particle buffers
// each sort.
static int64_t graph_period(const pc_column* h)
{
    auto lcm = [](int64_t a, int64_t b) { return a / gcd64(a, b) * b; };
    int64_t p = lcm(2, 2 * int64_t(h->cfg.ion_subcycle));
    if (h->cfg.sort_interval > 0) p = lcm(p, 2 * kIonSortEvery * int64_t(h->cfg.sort_interval));
    return p;
}

static void drop_graph(pc_column* h)
{
    for (pc_column::Graph& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

// cached graphs per column: whole periods for every phase a run starts at
// plus the shorter remainders of step counts that are not whole periods
constexpr size_t kMaxGraphs = 64;

// Capture `len` steps from the current bookkeeping state into a graph (host
// bookkeeping is restored: nothing executes during capture).  On a stream
// that cannot be captured the column stays eager (use_graphs = 0).
static pc_status capture_steps(pc_column* h, int64_t len, const int64_t key[6], hipGraphExec_t* out)
{
    *out = nullptr;
    const int64_t step = h->step;
    const int re = h->re_cur, ri = h->ri_cur, c0 = h->cur[0], c1 = h->cur[1];
    hipError_t e = hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->use_graphs = 0;   // e.g. the legacy default stream: stay eager
        return PC_OK;
    }
    pc_status st = PC_OK;
    for (int64_t k = 0; k < len && st == PC_OK; ++k) st = enqueue_step(h, false, 0);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->st, &g);
    h->step = step;
    h->re_cur = re;
    h->ri_cur = ri;
    h->cur[0] = c0;
    h->cur[1] = c1;
    if (st != PC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if (h->graphs.size() >= kMaxGraphs) {   // evict the least recently used
        size_t old = 0;
        for (size_t k = 1; k < h->graphs.size(); ++k)
            if (h->graphs[k].used < h->graphs[old].used) old = k;
        (void)hipGraphExecDestroy(h->graphs[old].exec);
        h->graphs.erase(h->graphs.begin() + old);
    }
    pc_column::Graph G;
    std::memcpy(G.key, key, sizeof(G.key));
    G.exec = x;
    G.used = ++h->graph_clock;
    h->graphs.push_back(G);
    *out = x;
    return PC_OK;
}

// Walk n_steps from the current bookkeeping state: whole periods and the
// remainder each as one graph (captured when missing), launched if
// `execute`, else only captured (the bookkeeping is then restored).  Steps
// that cannot be replayed run eagerly (execute) or are skipped (prepare).
static pc_status walk_steps(pc_column* h, int64_t n_steps, bool execute)
{
    const int64_t period = graph_period(h);
    const bool timer_on = !h->tev.empty();
    const int64_t tcap = int64_t(h->tev.size() / 2);
    // graph replay needs a capturable (non-null) stream; event buffers and the
    // kernel timer run eagerly (graph-recorded events have no readable time)
    const bool graphs = h->use_graphs && h->st != nullptr && !h->ev[0] && !h->ev[1] &&
                        period <= 4096 && !timer_on;
    const int64_t step0 = h->step;
    const int re0 = h->re_cur, ri0 = h->ri_cur, c00 = h->cur[0], c10 = h->cur[1];
    pc_status s = PC_OK;
    int64_t left = n_steps;
    while (left > 0 && s == PC_OK) {
        if (graphs && h->use_graphs) {
            const int64_t len = left >= period ? period : left;
            const int64_t key[6] = {h->step % period, h->re_cur, h->ri_cur, h->cur[0], h->cur[1], len};
            hipGraphExec_t x = nullptr;
            for (pc_column::Graph& g : h->graphs)
                if (std::memcmp(g.key, key, sizeof(key)) == 0) {
                    x = g.exec;
                    g.used = ++h->graph_clock;
                    break;
                }
            if (!x) {
                s = capture_steps(h, len, key, &x);
                if (s != PC_OK) break;
                if (!x) continue;   // capture unavailable: eager from now on
            }
            if (execute) {
                const hipError_t e = hipGraphLaunch(x, h->st);
                if (e != hipSuccess) {
                    s = hip_fail(e, "hipGraphLaunch");
                    break;
                }
            }
            for (int64_t k = 0; k < len && s == PC_OK; ++k) s = enqueue_step(h, false, 0, false);
            left -= len;
        } else if (execute) {
            const bool t = timer_on && h->tcount < tcap;
            s = enqueue_step(h, t, h->tcount);
            if (t) h->tcount += 1;
            left -= 1;
        } else {
            break;
        }
    }
    if (!execute) {
        h->step = step0;
        h->re_cur = re0;
        h->ri_cur = ri0;
        h->cur[0] = c00;
        h->cur[1] = c10;
    }
    return s;
}

pc_status pc_step(pc_handle h, int64_t n_steps)
{
    if (!h || n_steps < 0) return fail(PC_ERR_INVALID_ARG, "bad handle or step count");
    if (h->batch_member) return fail(PC_ERR_INVALID_ARG, "column belongs to a batch: step the batch");
    if (h->poisoned) return fail(PC_ERR_POISONED, "an earlier device error is pending");
    if (h->slots_dirty) {   // pair sink: slot of every id of the current stores
        if (h->fp32) HIPCHK(pclaunch::slot_map(h->P, h->buf32[0][h->cur[0]], h->buf32[1][h->cur[1]], h->st));
        else HIPCHK(pclaunch::slot_map(h->P, soa_of(h, 0), soa_of(h, 1), h->st));
        h->slots_dirty = 0;
    }
    return walk_steps(h, n_steps, true);
}

pc_status pc_prepare_graphs(pc_handle h, int64_t n_steps)
{
    if (!h || n_steps < 0) return fail(PC_ERR_INVALID_ARG, "bad handle or step count");
    if (h->batch_member) return fail(PC_ERR_INVALID_ARG, "column belongs to a batch: step the batch");
    return walk_steps(h, n_steps, false);
}

pc_status pc_deposit(pc_handle h, const double* x, int64_t n, int64_t* rho)
{
    if (!h || !rho || n < 0 || (n > 0 && !x)) return fail(PC_ERR_INVALID_ARG, "bad deposit arguments");
    HIPCHK(pclaunch::deposit(h->P, x, n, rho, h->st));
    return PC_OK;
}

pc_status pc_solve_field(pc_handle h, const int64_t* rho_e, const int64_t* rho_i, double* phi, double* E)
{
    if (!h || !rho_e || !rho_i || !E) return fail(PC_ERR_INVALID_ARG, "bad field arguments");
    HIPCHK(pclaunch::field(h->P, rho_e, rho_i, E, phi, 0, h->st));
    return PC_OK;
}

pc_status pc_moments(pc_handle h, int32_t cells_per_group, int32_t reset_iz, int64_t* out)
{
    if (!h || !out || cells_per_group < 1) return fail(PC_ERR_INVALID_ARG, "bad moments arguments");
    const int64_t ng = (h->d.nc + cells_per_group - 1) / cells_per_group;
    const int64_t len = 7 * int64_t(h->d.nc) + ng * 240;
    if (h->fp32)
        HIPCHK(pclaunch::moments(h->P, h->buf32[0][h->cur[0]], h->buf32[1][h->cur[1]], cells_per_group, reset_iz,
                                 out, len, h->st));
    else
        HIPCHK(pclaunch::moments(h->P, soa_of(h, 0), soa_of(h, 1), cells_per_group, reset_iz, out, len, h->st));
    return PC_OK;
}

pc_status pc_get_counts(pc_handle h, pc_counts* out)
{
    if (!h || !out) return fail(PC_ERR_INVALID_ARG, "null argument");
    const pc_status s = read_counters(h);
    if (s != PC_OK) return s;
    for (int k = 0; k < 2; ++k) {
        out->n[k] = h->host_cnt.n[k];
        out->next_id[k] = h->host_cnt.next_id[k];
    }
    out->step = h->host_cnt.step;
    out->errors = h->host_cnt.err;
    out->pad = 0;
    out->births_last = h->host_cnt.births_last;
    out->births_since_ion = h->host_cnt.births_since_ion;
    out->V_anode = h->host_cnt.V;
    out->J_cond = h->host_cnt.J;
    out->vsum_ion = h->host_cnt.vsum_i;
    out->emit_carry = h->host_cnt.carry;
    return PC_OK;
}

pc_status pc_set_circuit(pc_handle h, double V_anode, int64_t vsum_ion, double emit_carry)
{
    if (!h || !(emit_carry >= 0.0 && emit_carry < 1.0) || !(V_anode == V_anode))
        return fail(PC_ERR_INVALID_ARG, "bad circuit state");
    pc_status s = read_counters(h);
    if (s != PC_OK) return s;
    h->host_cnt.V = V_anode;
    h->host_cnt.vsum_i = vsum_ion;
    h->host_cnt.carry = emit_carry;
    return write_counters(h);
}

pc_status pc_set_balance(pc_handle h, int64_t births_last, int64_t births_since_ion)
{
    if (!h || births_last < 0 || births_since_ion < 0) return fail(PC_ERR_INVALID_ARG, "bad ionization tallies");
    pc_status s = read_counters(h);
    if (s != PC_OK) return s;
    h->host_cnt.births_last = births_last;
    h->host_cnt.births_since_ion = births_since_ion;
    return write_counters(h);
}

pc_status pc_get_state(pc_handle h, int32_t species, double* x, double* vx, double* vy, double* vz, uint32_t* id,
                       int64_t cap)
{
    if (!h || (species != 0 && species != 1) || cap < 0) return fail(PC_ERR_INVALID_ARG, "bad state arguments");
    pc_status s = read_counters(h);
    if (s != PC_OK) return s;
    const int64_t n = std::min<int64_t>(cap, h->host_cnt.n[species]);
    if (n == 0) return PC_OK;
    if (h->fp32) {
        const pcdev::SoaIO dst{x, vx, vy, vz, id};
        HIPCHK(pclaunch::to64(h->P, h->buf32[species][h->cur[species]], dst, n, species, h->st));
        return PC_OK;
    }
    const Soa q = soa_of(h, species);
    if (x) HIPCHK(hipMemcpyAsync(x, q.x, n * 8, hipMemcpyDeviceToDevice, h->st));
    if (vx) HIPCHK(hipMemcpyAsync(vx, q.vx, n * 8, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(pclaunch::vt_split(q.vt, vy, vz, n, h->st));
    if (id) HIPCHK(hipMemcpyAsync(id, q.id, n * 4, hipMemcpyDeviceToDevice, h->st));
    return PC_OK;
}

pc_status pc_set_state(pc_handle h, int32_t species, int64_t n, const double* x, const double* vx,
                       const double* vy, const double* vz, const uint32_t* id)
{
    if (!h || (species != 0 && species != 1) || n < 0) return fail(PC_ERR_INVALID_ARG, "bad state arguments");
    if (n > h->d.cap) return fail(PC_ERR_CAPACITY, "state larger than the particle capacity");
    if (n > 0 && (!x || !vx || !vy || !vz || !id)) return fail(PC_ERR_INVALID_ARG, "null state array");
    pc_status s = read_counters(h);
    if (s != PC_OK) return s;
    const Soa q = soa_of(h, species);
    if (!h->fp32 && n > 0) {
        HIPCHK(hipMemcpyAsync(q.x, x, n * 8, hipMemcpyDeviceToDevice, h->st));
        HIPCHK(hipMemcpyAsync(q.vx, vx, n * 8, hipMemcpyDeviceToDevice, h->st));
        HIPCHK(pclaunch::vt_join(vy, vz, q.vt, n, h->st));
        HIPCHK(hipMemcpyAsync(q.id, id, n * 4, hipMemcpyDeviceToDevice, h->st));
    }
    h->host_cnt.n[species] = n;
    h->host_cnt.err = 0;
    h->slots_dirty = h->d.pair;
    h->host_cnt.nb = 0;
    h->host_cnt.nh[0] = h->host_cnt.nh[1] = 0;
    if ((s = write_counters(h)) != PC_OK) return s;
    // positions must lie in [0, L): checked by a deposit into scratch charge
    // (the FP32 conversion checks them itself)
    if (n > 0 && h->fp32) {
        const pcdev::SoaIO src{const_cast<double*>(x), const_cast<double*>(vx), const_cast<double*>(vy),
                               const_cast<double*>(vz), const_cast<uint32_t*>(id)};
        HIPCHK(pclaunch::from64(h->P, src, h->buf32[species][h->cur[species]], n, species, h->st));
    } else if (n > 0) {
        int64_t* scratch = h->rho[0][1 - h->re_cur];   // the next electron charge buffer: zero and unused
        HIPCHK(pclaunch::deposit(h->P, q.x, n, scratch, h->st));
        HIPCHK(pclaunch::fill_i64(scratch, h->d.nn, 0, h->st));
    }
    // the ions' charge is held between ion steps: it is the new ions' from now on
    if (species == 1) {
        int64_t* held = h->rho[1][h->ri_cur];
        HIPCHK(pclaunch::fill_i64(held, h->d.nn, 0, h->st));
        if (n > 0) {
            if (h->fp32) HIPCHK(pclaunch::deposit(h->P, h->buf32[1][h->cur[1]], n, held, h->st));
            else HIPCHK(pclaunch::deposit(h->P, q.x, n, held, h->st));
        }
    }
    if (n > 0) {
        if ((s = read_counters(h)) != PC_OK) return s;
        if (h->host_cnt.err) {
            h->poisoned = 1;
            return map_errors(h->host_cnt.err);
        }
    }
    h->poisoned = 0;
    return PC_OK;
}

pc_status pc_set_counters(pc_handle h, int64_t step, int64_t next_e, int64_t next_i)
{
    if (!h || step < 0 || next_e < 0 || next_i < 0 || step > 0xFFFFFFFFll || next_e > 0xFFFFFFFFll ||
        next_i > 0xFFFFFFFFll)
        return fail(PC_ERR_INVALID_ARG, "bad counters");
    pc_status s = read_counters(h);
    if (s != PC_OK) return s;
    h->host_cnt.step = step;
    h->host_cnt.next_id[0] = next_e;
    h->host_cnt.next_id[1] = next_i;
    if ((s = write_counters(h)) != PC_OK) return s;
    h->step = step;
    h->slots_dirty = h->d.pair;
    return PC_OK;
}

pc_status pc_get_field(pc_handle h, double* E, int64_t* rho_e, int64_t* rho_i)
{
    if (!h) return fail(PC_ERR_INVALID_ARG, "null handle");
    const int64_t nb = int64_t(h->d.nn) * 8;
    if (E) HIPCHK(hipMemcpyAsync(E, h->P.E, nb, hipMemcpyDeviceToDevice, h->st));
    if (rho_e) HIPCHK(hipMemcpyAsync(rho_e, h->rho[0][h->re_cur], nb, hipMemcpyDeviceToDevice, h->st));
    if (rho_i) HIPCHK(hipMemcpyAsync(rho_i, h->rho[1][h->ri_cur], nb, hipMemcpyDeviceToDevice, h->st));
    return PC_OK;
}

pc_status pc_set_field(pc_handle h, const double* E)
{
    if (!h || !E) return fail(PC_ERR_INVALID_ARG, "null argument");
    HIPCHK(hipMemcpyAsync(h->P.E, E, int64_t(h->d.nn) * 8, hipMemcpyDeviceToDevice, h->st));
    if (h->d.periodic) HIPCHK(hipMemcpyAsync(h->P.E + h->d.nc, E, 8, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(pclaunch::scale_field(h->P, h->st));
    return PC_OK;
}

pc_status pc_set_events(pc_handle h, uint8_t* ev_e, int64_t len_e, uint8_t* ev_i, int64_t len_i)
{
    if (!h || len_e < 0 || len_i < 0) return fail(PC_ERR_INVALID_ARG, "bad event buffers");
    if (h->batch_member) return fail(PC_ERR_INVALID_ARG, "batched steps record no events");
    drop_graph(h);
    h->ev[0] = ev_e;
    h->evlen[0] = ev_e ? len_e : 0;
    h->ev[1] = ev_i;
    h->evlen[1] = ev_i ? len_i : 0;
    return PC_OK;
}

pc_status pc_sync(pc_handle h)
{
    if (!h) return fail(PC_ERR_INVALID_ARG, "null handle");
    const pc_status s = read_counters(h);
    if (s != PC_OK) return s;
    if (h->host_cnt.err) {
        h->poisoned = 1;
        return map_errors(h->host_cnt.err);
    }
    return PC_OK;
}

pc_status pc_timer_enable(pc_handle h, int64_t max_launches)
{
    if (!h || max_launches < 0 || max_launches > (int64_t(1) << 24)) return fail(PC_ERR_INVALID_ARG, "bad timer size");
    if (h->batch_member) return fail(PC_ERR_INVALID_ARG, "time the batch, not a member column");
    HIPCHK(hipStreamSynchronize(h->st));
    drop_graph(h);
    for (hipEvent_t e : h->tev) HIPCHK(hipEventDestroy(e));
    h->tev.clear();
    h->tcount = 0;
    // timing only (read after the stream is synchronized): no system-scope
    // fence, whose cache writeback and invalidation at every recorded event
    // would slow the timed launch and the work after it
    for (int64_t k = 0; k < 2 * max_launches; ++k) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        h->tev.push_back(e);
    }
    return PC_OK;
}

pc_status pc_timer_read(pc_handle h, double* total_ms, int64_t* launches)
{
    if (!h || !total_ms || !launches) return fail(PC_ERR_INVALID_ARG, "null argument");
    HIPCHK(hipStreamSynchronize(h->st));
    double tot = 0.0;
    for (int64_t k = 0; k < h->tcount; ++k) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, h->tev[2 * k], h->tev[2 * k + 1]));
        tot += double(ms);
    }
    *total_ms = tot;
    *launches = h->tcount;
    h->tcount = 0;
    return PC_OK;
}

void pc_destroy(pc_handle h)
{
    if (!h || h->batch_member) return;   // members are released with their batch
    drop_graph(h);
    for (hipEvent_t e : h->tev) (void)hipEventDestroy(e);
    delete h;
}

const char* pc_status_string(pc_status s)
{
    switch (s) {
    case PC_OK: return "ok";
    case PC_ERR_INVALID_ARG: return "invalid argument";
    case PC_ERR_UNSTABLE_CONFIG: return "unstable configuration";
    case PC_ERR_CAPACITY: return "capacity exceeded";
    case PC_ERR_NONFINITE: return "non-finite or out-of-range value";
    case PC_ERR_ECAP: return "electron energy above the collision bound";
    case PC_ERR_GCAP: return "ion relative speed above the collision bound";
    case PC_ERR_HIP: return "HIP runtime error";
    case PC_ERR_POISONED: return "handle poisoned by an earlier device error";
    case PC_ERR_WORKSPACE: return "workspace too small or misaligned";
    case PC_ERR_IDS: return "particle id space exhausted";
    default: return "unknown status";
    }
}

const char* pc_last_error(void) { return g_last_error.c_str(); }

pc_status pc_stream_probe(const double* src, double* dst, int64_t n, int32_t blocks, void* hip_stream)
{
    if (n < 0 || n > (int64_t(1) << 29) || (n > 0 && (!src || !dst)) || blocks < 0 || blocks > 65536)
        return fail(PC_ERR_INVALID_ARG, "stream probe: 0 <= n <= 2^29, non-null arrays, blocks <= 65536");
    HIPCHK(pclaunch::stream_copy(src, dst, n, blocks > 0 ? blocks : 4096, static_cast<hipStream_t>(hip_stream)));
    return PC_OK;
}

}  // extern "C"

// ===================================================================== batch
// Many independent columns advanced together: one launch per phase covers
// every column (particle chunks of all columns, then one finish workgroup
// per column), so small columns share the GPU instead of each leaving most
// of it idle.  Columns keep their own parameters, seeds, particle ids and
// buffers; a column stepped in a batch evolves exactly as it would alone.

using pcdev::BatchItem;
using pcdev::BatchStep;
using pcdev::ColumnDev;

namespace {
constexpr int kMinChunk = 256;   // smallest chunk (particles per workgroup) the tuner may pick
}

struct pc_batch {
    std::vector<pc_column*> cols;
    std::vector<int64_t> col_off;  // workspace offset of each column
    int fp32, S, K, chunk;
    hipStream_t st;
    ColumnDev* dcols;
    BatchItem* ditems[2];
    int64_t items_cap;
    int n_items[2];
    int64_t step;
    int cur[2], re_cur, ri_cur;
    int poisoned;
    int use_graphs;
    hipGraphExec_t gexec;
    int64_t gkey[7];
    std::vector<hipEvent_t> tev;   // timer pool: 2 events per electron push launch
    int64_t tcount;
};

namespace {

struct BatchLayout {
    int64_t cols, items[2], items_cap, total;
    std::vector<int64_t> col_off;
};

pc_status batch_layout(const pc_config* cfgs, int32_t n, std::vector<Derived>& ds, BatchLayout& BL)
{
    if (!cfgs || n < 1 || n > 65535) return fail(PC_ERR_INVALID_ARG, "batch needs 1..65535 column configs");
    ds.resize(n);
    for (int32_t c = 0; c < n; ++c) {
        const pc_status s = derive(&cfgs[c], &ds[c]);
        if (s != PC_OK) return fail(s, "column " + std::to_string(c) + ": " + g_last_error);
        if (cfgs[c].precision != cfgs[0].precision)
            return fail(PC_ERR_INVALID_ARG, "batch columns must share one precision");
        if (cfgs[c].ion_subcycle != cfgs[0].ion_subcycle)
            return fail(PC_ERR_INVALID_ARG, "batch columns must share one ion subcycle");
        if (cfgs[c].sort_interval != cfgs[0].sort_interval)
            return fail(PC_ERR_INVALID_ARG, "batch columns must share one sort interval");
        if (cfgs[c].wall_mode == PC_WALL_PAIR)
            return fail(PC_ERR_INVALID_ARG, "the pair sink runs on single columns only");
        if (cfgs[c].emit_J > 0.0 || cfgs[c].circuit_R > 0.0)
            return fail(PC_ERR_INVALID_ARG, "cathode emission and the circuit run on single columns only");
    }
    int64_t items = 0;
    for (int32_t c = 0; c < n; ++c) items += (ds[c].cap + kMinChunk - 1) / kMinChunk;
    if (items > (int64_t(1) << 31) - 1) return fail(PC_ERR_INVALID_ARG, "too many particle chunks");
    int64_t o = 0;
    BL.cols = o;
    o = align256(o + int64_t(n) * int64_t(sizeof(ColumnDev)));
    for (int s = 0; s < 2; ++s) {
        BL.items[s] = o;
        o = align256(o + items * int64_t(sizeof(BatchItem)));
    }
    BL.items_cap = items;
    BL.col_off.resize(n);
    for (int32_t c = 0; c < n; ++c) {
        BL.col_off[c] = o;
        o = align256(o + layout(ds[c]).total);
    }
    BL.total = o;
    return PC_OK;
}

// item tables for one chunk size: every column's chunks, column by column
pc_status upload_items(pc_batch* b, int chunk)
{
    std::vector<BatchItem> it[2];
    for (size_t c = 0; c < b->cols.size(); ++c) {
        const int64_t cap = b->cols[c]->d.cap;
        const int nk = int(std::max<int64_t>(1, (cap + chunk - 1) / chunk));
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < nk; ++k) it[s].push_back(BatchItem{int32_t(c), k, nk, 0});
    }
    for (int s = 0; s < 2; ++s) {
        if (int64_t(it[s].size()) > b->items_cap) return fail(PC_ERR_INVALID_ARG, "chunk below the minimum");
        HIPCHK(hipMemcpyAsync(b->ditems[s], it[s].data(), it[s].size() * sizeof(BatchItem), hipMemcpyHostToDevice,
                              b->st));
        b->n_items[s] = int(it[s].size());
    }
    HIPCHK(hipStreamSynchronize(b->st));
    b->chunk = chunk;
    return PC_OK;
}

void batch_drop_graph(pc_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
}

// the members' host bookkeeping follows the batch
void batch_publish(pc_batch* b)
{
    for (pc_column* h : b->cols) {
        h->step = b->step;
        h->re_cur = b->re_cur;
        h->ri_cur = b->ri_cur;
        h->cur[0] = b->cur[0];
        h->cur[1] = b->cur[1];
        h->cfg.sort_interval = b->K;
    }
}

pc_status enqueue_batch_step(pc_batch* b, bool time_it, int64_t slot)
{
    const bool ion = b->step % b->S == 0;
    BatchStep bs{};
    bs.cur[0] = b->cur[0];
    bs.cur[1] = b->cur[1];
    bs.re_new = 1 - b->re_cur;
    bs.re_old = b->re_cur;
    bs.ri_use = ion ? 1 - b->ri_cur : b->ri_cur;
    bs.ri_old = ion ? b->ri_cur : -1;
    bs.ion = ion;
    const int n = int(b->cols.size());
    hipEvent_t t0 = time_it ? b->tev[2 * slot] : nullptr, t1 = time_it ? b->tev[2 * slot + 1] : nullptr;
    HIPCHK(pclaunch::batch_push_e(b->dcols, b->fp32, b->ditems[0], b->n_items[0], bs, b->st, t0, t1));
    if (ion) HIPCHK(pclaunch::batch_advance_i(b->dcols, b->fp32, b->ditems[1], b->n_items[1], bs, b->st));
    HIPCHK(pclaunch::batch_finish(b->dcols, n, b->fp32, bs, b->st));
    b->re_cur = 1 - b->re_cur;
    if (ion) b->ri_cur = 1 - b->ri_cur;
    b->step += 1;
    if (b->K > 0 && b->step % b->K == 0) {
        const bool ions = b->step % (int64_t(b->K) * kIonSortEvery) == 0;
        for (int s = 0; s < (ions ? 2 : 1); ++s) {
            HIPCHK(pclaunch::batch_sort(b->dcols, n, b->fp32, s, b->ditems[s], b->n_items[s], b->cur[s], b->st));
            b->cur[s] = 1 - b->cur[s];
        }
    }
    return PC_OK;
}

int64_t batch_period(const pc_batch* b)
{
    auto lcm = [](int64_t a, int64_t c) { return a / gcd64(a, c) * c; };
    int64_t p = lcm(2, 2 * int64_t(b->S));
    if (b->K > 0) p = lcm(p, 2 * kIonSortEvery * int64_t(b->K));
    return p;
}

pc_status capture_batch(pc_batch* b, int64_t period)
{
    const int64_t step = b->step;
    const int re = b->re_cur, ri = b->ri_cur, c0 = b->cur[0], c1 = b->cur[1];
    batch_drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b->use_graphs = 0;
        return PC_OK;
    }
    pc_status st = PC_OK;
    for (int64_t k = 0; k < period && st == PC_OK; ++k) st = enqueue_batch_step(b, false, 0);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->st, &g);
    b->step = step;
    b->re_cur = re;
    b->ri_cur = ri;
    b->cur[0] = c0;
    b->cur[1] = c1;
    if (st != PC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->gexec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    const int64_t key[7] = {step % period, re, ri, c0, c1, b->K, b->chunk};
    std::memcpy(b->gkey, key, sizeof(key));
    return PC_OK;
}

}  // namespace

extern "C" {

pc_status pc_query_batch_sizes(const pc_config* cfgs, int32_t n_columns, int64_t* workspace_bytes)
{
    if (!workspace_bytes) return fail(PC_ERR_INVALID_ARG, "null output");
    std::vector<Derived> ds;
    BatchLayout BL;
    const pc_status s = batch_layout(cfgs, n_columns, ds, BL);
    if (s != PC_OK) return s;
    *workspace_bytes = BL.total;
    return PC_OK;
}

pc_status pc_init_batch(const pc_config* cfgs, int32_t n_columns, void* workspace, size_t bytes, void* hip_stream,
                        pc_batch_handle* out)
{
    if (!out || !workspace) return fail(PC_ERR_INVALID_ARG, "null workspace or handle");
    *out = nullptr;
    std::vector<Derived> ds;
    BatchLayout BL;
    pc_status s = batch_layout(cfgs, n_columns, ds, BL);
    if (s != PC_OK) return s;
    if (int64_t(bytes) < BL.total) return fail(PC_ERR_WORKSPACE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) & 255u) return fail(PC_ERR_WORKSPACE, "workspace not 256-byte aligned");
    pc_batch* b = new (std::nothrow) pc_batch();
    if (!b) return fail(PC_ERR_INVALID_ARG, "host allocation failed");
    char* base = static_cast<char*>(workspace);
    b->st = static_cast<hipStream_t>(hip_stream);
    b->fp32 = ds[0].fp32;
    b->S = cfgs[0].ion_subcycle;
    b->K = cfgs[0].sort_interval;
    b->dcols = reinterpret_cast<ColumnDev*>(base + BL.cols);
    b->ditems[0] = reinterpret_cast<BatchItem*>(base + BL.items[0]);
    b->ditems[1] = reinterpret_cast<BatchItem*>(base + BL.items[1]);
    b->items_cap = BL.items_cap;
    b->col_off = BL.col_off;
    b->use_graphs = 1;
    auto cleanup = [&](pc_status st) {
        for (pc_column* h : b->cols) {
            h->batch_member = 0;
            pc_destroy(h);
        }
        delete b;
        return st;
    };
    std::vector<ColumnDev> table(n_columns);
    for (int32_t c = 0; c < n_columns; ++c) {
        pc_column* h = nullptr;
        s = column_init(&cfgs[c], ds[c], base + BL.col_off[c], b->st, &h);
        if (s != PC_OK) return cleanup(fail(s, "column " + std::to_string(c) + ": " + g_last_error));
        h->batch_member = 1;
        h->use_graphs = 0;
        b->cols.push_back(h);
        ColumnDev& C = table[c];
        C.P = h->P;
        for (int sp = 0; sp < 2; ++sp)
            for (int k = 0; k < 2; ++k) {
                C.soa[sp][k] = h->buf[sp][k];
                C.soa32[sp][k] = h->buf32[sp][k];
                C.rho[sp][k] = h->rho[sp][k];
            }
    }
    // every column starts from the same bookkeeping state (one sort at init if K > 0)
    b->step = 0;
    b->re_cur = b->cols[0]->re_cur;
    b->ri_cur = b->cols[0]->ri_cur;
    b->cur[0] = b->cols[0]->cur[0];
    b->cur[1] = b->cols[0]->cur[1];
    hipError_t e = hipMemcpyAsync(b->dcols, table.data(), table.size() * sizeof(ColumnDev), hipMemcpyHostToDevice,
                                  b->st);
    if (e != hipSuccess) return cleanup(hip_fail(e, "pc_init_batch table"));
    const int64_t mean_cap = [&] {
        int64_t t = 0;
        for (const Derived& d : ds) t += d.cap;
        return t / n_columns;
    }();
    // default chunk: about four workgroups per 1024 particles of the mean column, within [1024, 4096]
    const int chunk = int(std::min<int64_t>(4096, std::max<int64_t>(1024, mean_cap / 256)));
    if ((s = upload_items(b, chunk)) != PC_OK) return cleanup(s);
    batch_publish(b);
    *out = b;
    return PC_OK;
}

pc_status pc_batch_step(pc_batch_handle b, int64_t n_steps)
{
    if (!b || n_steps < 0) return fail(PC_ERR_INVALID_ARG, "bad handle or step count");
    if (b->poisoned) return fail(PC_ERR_POISONED, "an earlier device error is pending");
    const int64_t period = batch_period(b);
    const bool timer_on = !b->tev.empty();
    const int64_t tcap = int64_t(b->tev.size() / 2);
    const bool graphs = b->use_graphs && b->st != nullptr && period <= 4096 && !timer_on;
    int64_t left = n_steps;
    pc_status s = PC_OK;
    while (left > 0 && s == PC_OK) {
        if (graphs && b->use_graphs && left >= period) {
            const int64_t key[7] = {b->step % period, b->re_cur, b->ri_cur, b->cur[0], b->cur[1], b->K, b->chunk};
            if (!b->gexec || std::memcmp(key, b->gkey, sizeof(key)) != 0) {
                s = capture_batch(b, period);
                if (s != PC_OK || !b->gexec) continue;
            }
            const hipError_t e = hipGraphLaunch(b->gexec, b->st);
            if (e != hipSuccess) s = hip_fail(e, "hipGraphLaunch");
            b->step += period;
            left -= period;
        } else {
            const bool t = timer_on && b->tcount < tcap;
            s = enqueue_batch_step(b, t, b->tcount);
            if (t) b->tcount += 1;
            left -= 1;
        }
    }
    batch_publish(b);
    return s;
}

pc_status pc_batch_column(pc_batch_handle b, int32_t column, pc_handle* out)
{
    if (!b || !out || column < 0 || column >= int32_t(b->cols.size()))
        return fail(PC_ERR_INVALID_ARG, "bad batch column");
    *out = b->cols[column];
    return PC_OK;
}

pc_status pc_batch_sync(pc_batch_handle b)
{
    if (!b) return fail(PC_ERR_INVALID_ARG, "null handle");
    HIPCHK(hipStreamSynchronize(b->st));
    for (size_t c = 0; c < b->cols.size(); ++c) {
        const pc_status s = pc_sync(b->cols[c]);
        if (s != PC_OK) {
            b->poisoned = 1;
            return fail(s, "column " + std::to_string(c) + ": " + g_last_error);
        }
    }
    return PC_OK;
}

pc_status pc_batch_get_tuning(pc_batch_handle b, pc_tuning* out)
{
    if (!b || !out) return fail(PC_ERR_INVALID_ARG, "null argument");
    out->chunk = b->chunk;
    out->sort_interval = b->K;
    out->n_items_e = b->n_items[0];
    out->n_items_i = b->n_items[1];
    out->us_per_step = 0.0;
    return PC_OK;
}

pc_status pc_batch_set_tuning(pc_batch_handle b, int32_t chunk, int32_t sort_interval)
{
    if (!b || chunk < kMinChunk || chunk > (1 << 24) || sort_interval < 0)
        return fail(PC_ERR_INVALID_ARG, "bad tuning");
    batch_drop_graph(b);
    if (chunk != b->chunk) {
        const pc_status s = upload_items(b, chunk);
        if (s != PC_OK) return s;
    }
    b->K = sort_interval;
    batch_publish(b);
    return PC_OK;
}

// Time trial_steps real steps per (chunk, sort interval) candidate and keep
// the fastest.  Neither setting changes any result: particle order affects
// no draw, deposit or field value.
pc_status pc_batch_tune(pc_batch_handle b, int32_t trial_steps, pc_tuning* out)
{
    if (!b || trial_steps < 1) return fail(PC_ERR_INVALID_ARG, "bad tuning arguments");
    static const int chunks[] = {1024, 2048, 3072, 4096, 6144, 8192};
    static const int sorts[] = {10, 20, 40, 80};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = 1e300;
    int bc = b->chunk, bk = b->K;
    pc_status s = PC_OK;
    for (int ci = 0; ci < int(sizeof(chunks) / sizeof(chunks[0])) && s == PC_OK; ++ci)
        for (int ki = -1; ki < 4 && s == PC_OK; ++ki) {
            if ((s = pc_batch_set_tuning(b, chunks[ci], sorts[ki < 0 ? 0 : ki])) != PC_OK) break;
            hipError_t e = hipEventRecord(e0, b->st);
            if (e == hipSuccess) s = pc_batch_step(b, trial_steps);
            if (s == PC_OK && e == hipSuccess) e = hipEventRecord(e1, b->st);
            if (s == PC_OK && e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (s == PC_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) s = hip_fail(e, "pc_batch_tune timing");
            if (s == PC_OK && ki >= 0 && ms < best) {   // ki < 0: warm-up of this chunk size
                best = ms;
                bc = chunks[ci];
                bk = sorts[ki];
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != PC_OK) return s;
    if ((s = pc_batch_set_tuning(b, bc, bk)) != PC_OK) return s;
    if ((s = pc_batch_sync(b)) != PC_OK) return s;
    if (out) {
        (void)pc_batch_get_tuning(b, out);
        out->us_per_step = best * 1e3 / double(trial_steps);
    }
    return PC_OK;
}

pc_status pc_batch_timer_enable(pc_batch_handle b, int64_t max_launches)
{
    if (!b || max_launches < 0 || max_launches > (int64_t(1) << 24)) return fail(PC_ERR_INVALID_ARG, "bad timer size");
    HIPCHK(hipStreamSynchronize(b->st));
    batch_drop_graph(b);
    for (hipEvent_t e : b->tev) HIPCHK(hipEventDestroy(e));
    b->tev.clear();
    b->tcount = 0;
    for (int64_t k = 0; k < 2 * max_launches; ++k) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));   // timing only, as above
        b->tev.push_back(e);
    }
    return PC_OK;
}

pc_status pc_batch_timer_read(pc_batch_handle b, double* total_ms, int64_t* launches)
{
    if (!b || !total_ms || !launches) return fail(PC_ERR_INVALID_ARG, "null argument");
    HIPCHK(hipStreamSynchronize(b->st));
    double tot = 0.0;
    for (int64_t k = 0; k < b->tcount; ++k) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, b->tev[2 * k], b->tev[2 * k + 1]));
        tot += double(ms);
    }
    *total_ms = tot;
    *launches = b->tcount;
    b->tcount = 0;
    return PC_OK;
}

void pc_batch_destroy(pc_batch_handle b)
{
    if (!b) return;
    batch_drop_graph(b);
    for (hipEvent_t e : b->tev) (void)hipEventDestroy(e);
    for (pc_column* h : b->cols) {
        h->batch_member = 0;
        pc_destroy(h);
    }
    delete b;
}

}  // extern "C"
