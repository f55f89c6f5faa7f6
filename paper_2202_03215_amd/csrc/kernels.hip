// kernels.hip -- gfx950 kernels of the 1D PIC-MCC column step.
//
// Layout: structure-of-arrays FP64 particles (x, vx, vy, vz, id) per species,
// int64 fixed-point node charges, FP64 node field.  One wave64 lane per
// particle; blocks take contiguous chunks of the (periodically cell-sorted)
// particle array so that a block's particles cover a narrow window of nodes,
// which is staged in LDS for the deposit.
#include "device.h"
#include "launch.h"
#include <hip/hip_ext.h>

namespace pcdev {

constexpr int kAdvBlock = 256;   // threads per block of the particle kernels
constexpr int kWindow = 256;     // LDS deposit window (nodes) per block
constexpr int kHalo = 64;        // window starts this many nodes before the chunk
constexpr int kOneBlock = 1024;  // threads of the single-workgroup kernels
constexpr int kMaxSeg = 8;       // nodes per thread in the field solve (n_nodes <= 8192)

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}

// DPP wavefront reductions and inclusive scans from the device library (all
// lanes participate; fixed combination order, hence deterministic)
extern "C" __device__ uint64_t __ockl_wfred_add_u64(uint64_t);
extern "C" __device__ double __ockl_wfred_add_f64(double);
extern "C" __device__ long __ockl_wfscan_add_i64(long, bool);
extern "C" __device__ double __ockl_wfscan_add_f64(double, bool);

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) { return __ockl_wfscan_add_i64(long(v), true); }
__device__ __forceinline__ double wave_incl_scan(double v) { return __ockl_wfscan_add_f64(v, true); }

__device__ __forceinline__ void set_err(const Params& P, uint32_t bits) { atomicOr(&P.cnt->err, bits); }

// ---------------------------------------------------------------- deposit
// add one node contribution: LDS window if inside, else global atomic
__device__ __forceinline__ void add_node(unsigned long long* win, int wbase, int64_t* rho, int node,
                                         int64_t v)
{
    // distinct scopes keep the two adds apart (an LDS add and a global add,
    // rather than one flat atomic through a selected address)
    const uint32_t li = uint32_t(node - wbase);
    if (li < uint32_t(kWindow))
        __hip_atomic_fetch_add(&win[li], (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        __hip_atomic_fetch_add((unsigned long long*)&rho[node], (unsigned long long)v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-aggregated CIC deposit.  The wave's two leading cells (those of the
// first pending lane and of the first lane outside that cell) are reduced
// together: weights of the first cell in the low 32 bits, of the second in
// the high 32 bits of one 64-bit DPP reduction (each sum <= 64 * 2^25 < 2^32,
// so no carry crosses).  Node j of a cell receives count * 2^25 minus the
// summed weights, node j+1 the summed weights.  Lanes in further cells
// deposit one by one.  Integer sums: the result is independent of order.
__device__ __forceinline__ void deposit_wave(const Params& P, unsigned long long* win, int wbase,
                                             int64_t* rho, bool alive, int j, int64_t a)
{
    const uint64_t m = __ballot(alive);
    if (m == 0) return;
    const int l1 = __ffsll((unsigned long long)m) - 1;
    const int j1 = __builtin_amdgcn_readlane(j, l1);
    const bool in1 = alive && j == j1;
    const uint64_t m1 = __ballot(in1);
    const uint64_t rest = m & ~m1;
    int l2 = 64, j2 = -1;
    if (rest != 0) {
        l2 = __ffsll((unsigned long long)rest) - 1;
        j2 = __builtin_amdgcn_readlane(j, l2);
    }
    const bool in2 = alive && !in1 && j == j2;
    const uint64_t m2 = __ballot(in2);
    const uint64_t packed = in1 ? uint64_t(a) : (in2 ? uint64_t(a) << 32 : 0ull);
    const uint64_t sum = __ockl_wfred_add_u64(packed);
    if (lane_id() == l1) {
        const int64_t s1 = int64_t(sum & 0xFFFFFFFFull), s2 = int64_t(sum >> 32);
        const int64_t c1 = int64_t(__popcll((unsigned long long)m1)) * kUnit;
        const int64_t c2 = int64_t(__popcll((unsigned long long)m2)) * kUnit;
        int n1 = j1 + 1;
        if (P.periodic && n1 == P.nc) n1 = 0;
        if (m2 == 0) {
            add_node(win, wbase, rho, j1, c1 - s1);
            add_node(win, wbase, rho, n1, s1);
        } else {
            int n2 = j2 + 1;
            if (P.periodic && n2 == P.nc) n2 = 0;
            if (n1 == j2) {            // adjacent cells share node j1 + 1
                add_node(win, wbase, rho, j1, c1 - s1);
                add_node(win, wbase, rho, n1, s1 + c2 - s2);
                add_node(win, wbase, rho, n2, s2);
            } else if (n2 == j1) {
                add_node(win, wbase, rho, j2, c2 - s2);
                add_node(win, wbase, rho, j1, s2 + c1 - s1);
                add_node(win, wbase, rho, n1, s1);
            } else {
                add_node(win, wbase, rho, j1, c1 - s1);
                add_node(win, wbase, rho, n1, s1);
                add_node(win, wbase, rho, j2, c2 - s2);
                add_node(win, wbase, rho, n2, s2);
            }
        }
    }
    if (alive && !in1 && !in2) {
        int j1n = j + 1;
        if (P.periodic && j1n == P.nc) j1n = 0;
        add_node(win, wbase, rho, j, kUnit - a);
        add_node(win, wbase, rho, j1n, a);
    }
}

// append the flagged lanes to a global list with one atomic per wave;
// returns the lane's list position or -1
__device__ __forceinline__ int64_t wave_append(bool flag, int64_t* counter)
{
    const uint64_t m = __ballot(flag);
    if (m == 0) return -1;
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader)
        base = atomicAdd((unsigned long long*)counter, (unsigned long long)__popcll((unsigned long long)m));
    base = __shfl(base, leader);
    return flag ? int64_t(base) + int64_t(lanes_below(m)) : -1;
}

// Conduction-current sums of the external circuit (section V): v_x of the
// particles alive after their push, truncated to 2^-20 m/s units, so that
// the sum does not depend on the order of the atomics.  Each lane sums its
// particles over the chunk, each wave adds its total to one of kCurSlots
// slots (spread so that waves do not queue on one address); the finish
// kernel adds the slots up.
constexpr int kCurSlots = 64;
__device__ __forceinline__ int64_t vunits(double v) { return int64_t(v * 1048576.0); }
__device__ __forceinline__ void add_current(int64_t* slots, int64_t lane_sum)
{
    const uint64_t t = __ockl_wfred_add_u64(uint64_t(lane_sum));
    const int slot = (int(blockIdx.x) * (kAdvBlock / 64) + int(threadIdx.x >> 6)) & (kCurSlots - 1);
    if (lane_id() == 0 && t != 0ull) atomicAdd((unsigned long long*)&slots[slot], (unsigned long long)t);
}

// contiguous chunk kb of nb equal (64-aligned) chunks of a particle array
__device__ __forceinline__ void chunk_range(int64_t n, int kb, int nb, int64_t& beg, int64_t& end)
{
    const int64_t per = ((n + nb - 1) / nb + 63) & ~int64_t(63);
    beg = int64_t(kb) * per;
    end = beg + per < n ? beg + per : n;
}

// Global access through a wave-uniform base and a 32-bit byte offset (each
// particle field stays below 4 GiB: capacity <= 2^29), which selects the
// scalar-base form of the vector load and store instructions instead of
// per-lane 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ T ld32(const T* __restrict__ base, uint32_t i)
{
    return *(const T*)((const char*)base + i * uint32_t(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st32(T* __restrict__ base, uint32_t i, T v)
{
    *(T*)((char*)base + i * uint32_t(sizeof(T))) = v;
}

// Philox key words reloaded inside a particle loop: the empty asm makes them
// loop-variant, so the ten round keys are rebuilt with scalar adds in each
// iteration instead of being held (and spilled) across the loop.
__device__ __forceinline__ void loop_keys(const Params& P, uint32_t& k0, uint32_t& k1)
{
    k0 = P.key0;
    k1 = P.key1;
    asm volatile("" : "+s"(k0), "+s"(k1));
}

// periodic reinjection / absorbing walls; returns false if the particle left
__device__ __forceinline__ bool apply_boundary(const Params& P, double& x, uint8_t& code)
{
    if (P.periodic) {
        if (x >= P.L) x -= P.L;
        else if (x < 0.0) {
            x += P.L;
            if (x >= P.L) x = 0.0;
        }
        if (!(x >= 0.0 && x < P.L)) {
            set_err(P, kErrRange);
            x = 0.0;
        }
        return true;
    }
    if (x >= 0.0 && x < P.L) return true;
    if (!(x < 0.0 || x >= P.L)) set_err(P, kErrRange);
    code = kEvAbsorb;
    return false;
}

// --------------------------------------------------- particle-store access
// FP64 stores keep x [m] and v [m/s]; FP32 stores keep (cell, offset) and
// velocities in cells per step.  Collision arithmetic is FP64 for both.
__device__ __forceinline__ void load_v(const Params&, const Soa& s, uint32_t i, int, double& vx, double& vy,
                                       double& vz)
{
    vx = s.vx[i];
    const double2 t = s.vt[i];
    vy = t.x;
    vz = t.y;
}
__device__ __forceinline__ void load_v(const Params& P, const Soa32& s, uint32_t i, int sp, double& vx,
                                       double& vy, double& vz)
{
    const double k = sp == kElectron ? P.u2v_e : P.u2v_i;
    vx = double(s.vx[i]) * k;
    const float2 t = s.vt[i];
    vy = double(t.x) * k;
    vz = double(t.y) * k;
}
__device__ __forceinline__ void store_v(const Params&, const Soa& s, uint32_t i, int, double vx, double vy,
                                        double vz)
{
    s.vx[i] = vx;
    s.vt[i] = make_double2(vy, vz);
}
__device__ __forceinline__ void store_v(const Params& P, const Soa32& s, uint32_t i, int sp, double vx,
                                        double vy, double vz)
{
    const double k = sp == kElectron ? P.u2v_e : P.u2v_i;
    s.vx[i] = float(vx / k);
    s.vt[i] = make_float2(float(vy / k), float(vz / k));
}
// position key of a position x [m] for put_particle: x itself (FP64) or x / dx (FP32)
__device__ __forceinline__ double key_of_x(const Params&, const Soa&, double x) { return x; }
__device__ __forceinline__ double key_of_x(const Params& P, const Soa32&, double x) { return x * P.inv_dx; }
// position key of a particle: x [m] (FP64) or cell + offset (FP32, exact in FP64)
__device__ __forceinline__ double pos_key(const Params&, const Soa& s, uint32_t i) { return s.x[i]; }
__device__ __forceinline__ double pos_key(const Params&, const Soa32& s, uint32_t i)
{
    return double(s.cell[i]) + double(s.off[i]);
}
// cell and 25-bit weight of a position key
__device__ __forceinline__ int key_cell(const Params& P, const Soa&, double xk, int64_t& a)
{
    double f;
    const int j = cell_frac(P, xk, f);
    a = frac_units(f);
    return j;
}
__device__ __forceinline__ int key_cell(const Params& P, const Soa32&, double xk, int64_t& a)
{
    int c = int(xk);
    if (c > P.nc - 1) c = P.nc - 1;
    if (c < 0) c = 0;
    a = frac_units(float(xk - double(c)));
    return c;
}
__device__ __forceinline__ void move_particle(const Soa& sp, uint32_t dst, uint32_t src)
{
    sp.x[dst] = sp.x[src];
    sp.vx[dst] = sp.vx[src];
    sp.vt[dst] = sp.vt[src];
    sp.id[dst] = sp.id[src];
}
__device__ __forceinline__ void move_particle(const Soa32& sp, uint32_t dst, uint32_t src)
{
    sp.cell[dst] = sp.cell[src];
    sp.off[dst] = sp.off[src];
    sp.vx[dst] = sp.vx[src];
    sp.vt[dst] = sp.vt[src];
    sp.id[dst] = sp.id[src];
}
// one particle held in registers (the finish kernel's tail prefetch)
template <class St> struct PartRegs;
template <> struct PartRegs<Soa> {
    double x, vx;
    double2 vt;
    uint32_t id;
};
template <> struct PartRegs<Soa32> {
    int32_t cell;
    float off, vx;
    float2 vt;
    uint32_t id;
};
__device__ __forceinline__ PartRegs<Soa> load_part(const Soa& sp, uint32_t i)
{
    return PartRegs<Soa>{sp.x[i], sp.vx[i], sp.vt[i], sp.id[i]};
}
__device__ __forceinline__ PartRegs<Soa32> load_part(const Soa32& sp, uint32_t i)
{
    return PartRegs<Soa32>{sp.cell[i], sp.off[i], sp.vx[i], sp.vt[i], sp.id[i]};
}
__device__ __forceinline__ void store_part(const Soa& sp, uint32_t i, const PartRegs<Soa>& r)
{
    sp.x[i] = r.x;
    sp.vx[i] = r.vx;
    sp.vt[i] = r.vt;
    sp.id[i] = r.id;
}
__device__ __forceinline__ void store_part(const Soa32& sp, uint32_t i, const PartRegs<Soa32>& r)
{
    sp.cell[i] = r.cell;
    sp.off[i] = r.off;
    sp.vx[i] = r.vx;
    sp.vt[i] = r.vt;
    sp.id[i] = r.id;
}
// write a new particle at slot p from a position key and a velocity [m/s]
__device__ __forceinline__ void put_particle(const Params& P, const Soa& s, int64_t p, int, double xk,
                                             const double v[3], uint32_t id)
{
    s.x[p] = xk;
    s.vx[p] = v[0];
    s.vt[p] = make_double2(v[1], v[2]);
    s.id[p] = id;
}
__device__ __forceinline__ void put_particle(const Params& P, const Soa32& s, int64_t p, int sp, double xk,
                                             const double v[3], uint32_t id)
{
    int c = int(xk);
    if (c > P.nc - 1) c = P.nc - 1;
    s.cell[p] = c;
    s.off[p] = float(xk - double(c));
    store_v(P, s, uint32_t(p), sp, v[0], v[1], v[2]);
    s.id[p] = id;
}

// cell index of particle i
__device__ __forceinline__ int cell_at(const Params& P, const Soa& s, int64_t i)
{
    double f;
    return cell_frac(P, s.x[i], f);
}
__device__ __forceinline__ int cell_at(const Params&, const Soa32& s, int64_t i) { return s.cell[i]; }
__device__ __forceinline__ void copy_particle(const Soa& d, int64_t p, const Soa& s, int64_t i)
{
    d.x[p] = s.x[i];
    d.vx[p] = s.vx[i];
    d.vt[p] = s.vt[i];
    d.id[p] = s.id[i];
}
__device__ __forceinline__ void copy_particle(const Soa32& d, int64_t p, const Soa32& s, int64_t i)
{
    d.cell[p] = s.cell[i];
    d.off[p] = s.off[i];
    d.vx[p] = s.vx[i];
    d.vt[p] = s.vt[i];
    d.id[p] = s.id[i];
}

__device__ __forceinline__ uint64_t draw52(uint32_t lo, uint32_t hi) { return ((uint64_t(hi) << 32) | lo) >> 12; }

// -------------------------------------------------------- electron collide
// One collision candidate: choose the process with u1 nu_max against the
// cumulative collision frequencies (elastic, excitation, ionization, else
// null), then scatter.  Ionizations (rare) are listed with the parent's slot,
// position and energy; their kinematics run in the finish kernel.
template <bool EV, class St>
__device__ __forceinline__ void collide_one(const Params& P, const St& sp, uint8_t* __restrict__ ev,
                                            int64_t evlen, uint32_t step, bool act, uint32_t i, uint2 wcd)
{
    const uint32_t stream = kStreamElectronStep;
    bool born = false;
    uint32_t id = 0;
    int jn = 0;
    double x = 0.0, epsb = 0.0;
    if (act) {
        double vx, vy, vz;
        load_v(P, sp, i, kElectron, vx, vy, vz);
        id = sp.id[i];
        const double u1 = unif52(wcd.x, wcd.y);   // words 2, 3 of the step's block 0
        const double v2 = (vx * vx + vy * vy) + vz * vz;
        const double eps = P.c_eps * v2;
        const double v = sqrt(v2);
        if (eps > P.eps_cap) set_err(P, kErrECap);
        const double s_el = sigma_elastic(P, eps);
        const double s_ex = sigma_inelastic(eps, P.ex_U, P.sx4);
        const double s_iz = sigma_inelastic(eps, P.iz_U, P.si4);
        const double c1 = s_el * v * P.Ng;
        const double c2 = c1 + s_ex * v * P.Ng;
        const double c3 = c2 + s_iz * v * P.Ng;
        if (c3 > P.nu_max) set_err(P, kErrNuMax);
        const double R = u1 * P.nu_max;
        uint8_t code = kEvNull;
        if (R < c3) {
            if (R < c2) {
                WordStream ws(id, step, stream, P.key0, P.key1);
                double nx, ny, nz, vn;
                isotropic(ws, nx, ny, nz);
                if (R < c1) {
                    code = kEvElastic;
                    const double cosx = ((vx * nx + vy * ny) + vz * nz) / v;
                    const double fac = 1.0 - P.mr2 * (1.0 - cosx);
                    vn = v * sqrt(fac);
                } else {
                    code = kEvExcite;
                    vn = sqrt((eps - P.ex_U) / P.c_eps);
                }
                store_v(P, sp, i, kElectron, vn * nx, vn * ny, vn * nz);
            } else {
                code = kEvIonize;
                x = pos_key(P, sp, i);
                epsb = eps;
                int64_t a_unused;
                jn = key_cell(P, sp, x, a_unused);
                born = true;
            }
        }
        if (EV && int64_t(id) < evlen) ev[id] = code;
    }
    const int64_t bp = wave_append(born, &P.cnt->nb);
    if (bp >= 0) {
        if (bp < P.max_births) {
            Birth b;
            b.pid = id;
            b.slot = i;
            b.x = x;
            b.eps = epsb;
            b.vs[0] = 0.0; b.vs[1] = 0.0; b.vs[2] = 0.0;
            b.pad = 0.0;
            P.births[bp] = b;
            atomicAdd((unsigned long long*)&P.iz[jn], 1ull);
        } else {
            set_err(P, kErrBirths);
        }
    }
}

// ------------------------------------------------------------ electron push
// Streaming pass over all electrons: CIC gather, leapfrog push, boundary,
// radial sink, null-collision candidate test (u0 < P_null), fused
// fixed-point deposit.  Candidates are listed in the block's segment and
// collided in a second phase of the same block; collisions change only
// velocities, so the deposit of phase 1 is final.
template <bool EV>
__device__ __forceinline__ void push_e_chunk(const Params& P, const Soa& sp, int64_t* __restrict__ rho,
                                             uint8_t* __restrict__ ev, int64_t evlen, int kb, int nb)
{
    __shared__ unsigned long long win[kWindow];
    __shared__ int ncand;
    const int64_t n = P.cnt->n[kElectron];
    const uint32_t step = uint32_t(P.cnt->step);
    const uint64_t kw = sink_threshold(P, kElectron);
    int64_t beg, end;
    chunk_range(n, kb, nb, beg, end);
    if (beg >= end) return;

    // software pipeline: the next tile's loads are issued before this tile's
    // work, the first tile's before the block sets up its deposit window
    // (their latency overlaps that of the window's anchor)
    double px = 0.0, pvx = 0.0;
    uint32_t pid = 0;
    const uint32_t ue = uint32_t(end);
    {
        const uint32_t i = uint32_t(beg) + threadIdx.x;
        if (i < ue) {
            px = ld32(sp.x, i);
            pvx = ld32(sp.vx, i);
            pid = ld32(sp.id, i);
        }
    }
    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) win[k] = 0ull;
    if (threadIdx.x == 0) ncand = 0;
    double f0;
    const int wbase = cell_frac(P, sp.x[beg], f0) - kHalo;
    __syncthreads();
    const double* __restrict__ E = P.E;
    uint32_t* __restrict__ cl = P.cand + beg;   // this block's candidate segment
    uint2* __restrict__ cw = P.cand_w + beg;
    int64_t cur = 0;   // this lane's v_x sum (external circuit)
    for (uint32_t i0 = uint32_t(beg); i0 < ue; i0 += kAdvBlock) {
        const uint32_t i = i0 + threadIdx.x;
        const bool act = i < ue;
        bool alive = false, cand = false;
        int jn = 0;
        int64_t an = 0;
        uint2 wcd = make_uint2(0u, 0u);
        double x = px, vx = pvx;
        const uint32_t id = pid;
        if (i + kAdvBlock < ue) {
            px = ld32(sp.x, i + kAdvBlock);
            pvx = ld32(sp.vx, i + kAdvBlock);
            pid = ld32(sp.id, i + kAdvBlock);
        }
        if (act) {
            double f;
            const int j = cell_frac(P, x, f);
            const double e0 = ld32(E, uint32_t(j)), e1 = ld32(E, uint32_t(j) + 1u);
            const double Ex = e0 + f * (e1 - e0);
            vx = vx + P.qmdt_e * Ex;
            x = x + vx * P.dt;
            uint8_t code = kEvNone;
            alive = apply_boundary(P, x, code);
            if (alive) {
                uint32_t k0, k1;
                loop_keys(P, k0, k1);
                const U4 w = philox10(id, step, 0u, kStreamElectronStep, k0, k1);
                const uint64_t k = draw52(w.a, w.b);
                if (k >= kw) {
                    alive = false;
                    code = kEvWall;
                } else {
                    cand = k < P.kn_e;
                }
                wcd = make_uint2(w.c, w.d);
            }
            if (alive) {
                st32(sp.x, i, x);
                st32(sp.vx, i, vx);
                double fn;
                jn = cell_frac(P, x, fn);
                an = frac_units(fn);
            }
            if (EV && !cand && int64_t(id) < evlen) ev[id] = code;
        }
        const int64_t hp = wave_append(act && !alive, &P.cnt->nh[kElectron]);
        if (hp >= 0) {
            if (hp < P.max_holes) P.holes[kElectron][hp] = i;
            else set_err(P, kErrLosses);
        }
        {   // candidates: one LDS atomic per wave into the block's segment
            const uint64_t m = __ballot(cand);
            if (m != 0) {
                const int leader = __ffsll((unsigned long long)m) - 1;
                int base = 0;
                if (lane_id() == leader) base = atomicAdd(&ncand, __popcll((unsigned long long)m));
                base = __shfl(base, leader);
                if (cand) {
                    const uint32_t q = uint32_t(base) + lanes_below(m);
                    st32(cl, q, i);
                    st32(cw, q, wcd);
                }
            }
        }
        if (P.circuit && alive) cur += vunits(vx);
        deposit_wave(P, win, wbase, rho, alive, jn, an);
    }
    if (P.circuit) add_current(P.csum, cur);
    __syncthreads();
    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) {
        const unsigned long long v = win[k];
        if (v != 0ull) {
            const int node = wbase + k;
            if (node >= 0 && node < P.nn) atomicAdd((unsigned long long*)&rho[node], v);
        }
    }
    // phase 2: this block's collision candidates (their data is still hot)
    const int nc = ncand;
    for (int k0 = 0; k0 < nc; k0 += kAdvBlock) {
        const int k = k0 + int(threadIdx.x);
        collide_one<EV>(P, sp, ev, evlen, step, k < nc, k < nc ? cl[k] : 0u,
                        k < nc ? cw[k] : make_uint2(0u, 0u));
    }
}

// -------------------------------------------------------------- ion advance
// Charge-exchange candidates (u0 < P_cx) are listed during the streaming
// pass and exchanged in a second phase of the same block, with every lane
// busy: a candidate (P_cx well below 1 %) would otherwise hold its whole wave
// through the Maxwellian draw.  The exchange changes only velocities, so the
// pass's deposit is final.
__device__ __forceinline__ void list_candidate(bool cand, int* ncand, uint32_t* __restrict__ cl,
                                               uint2* __restrict__ cw, uint32_t i, uint2 wcd)
{
    const uint64_t m = __ballot(cand);
    if (m == 0) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(ncand, __popcll((unsigned long long)m));
    base = __shfl(base, leader);
    if (cand) {
        const uint32_t q = uint32_t(base) + lanes_below(m);
        st32(cl, q, i);
        st32(cw, q, wcd);
    }
}

// One charge-exchange candidate: a Maxwellian atom velocity a (three
// normals of the ion's step stream), accepted with probability g / g_cap for
// the relative speed g; the ion takes a.
template <bool EV, class St>
__device__ __forceinline__ void exchange_one(const Params& P, const St& sp, uint8_t* __restrict__ ev,
                                             int64_t evlen, uint32_t step, bool act, uint32_t i, uint2 wcd)
{
    if (!act) return;
    const uint32_t id = sp.id[i];
    const double u1 = unif52(wcd.x, wcd.y);
    double vx, vy, vz;
    load_v(P, sp, i, kIon, vx, vy, vz);
    WordStream ws(id, step, kStreamIonStep, P.key0, P.key1);
    double g0, g1, g2;
    normal3(ws, g0, g1, g2);
    const double ax = P.sig_a * g0, ay = P.sig_a * g1, az = P.sig_a * g2;
    const double dx = vx - ax, dy = vy - ay, dz = vz - az;
    const double g = sqrt((dx * dx + dy * dy) + dz * dz);
    if (g > P.g_cap) set_err(P, kErrGCap);
    uint8_t code = kEvNull;
    if (u1 * P.g_cap < g) {
        code = kEvCX;
        store_v(P, sp, i, kIon, ax, ay, az);
    }
    if (EV && int64_t(id) < evlen) ev[id] = code;
}

// Ions on subcycle steps (dt_i = S dt): gather, push, boundary, radial sink,
// charge exchange with a Maxwellian atom (null-collision bound Ng sigma g_cap,
// accepted with g / g_cap, the ion takes the atom's velocity), deposit.
template <bool EV>
__device__ __forceinline__ void advance_i_chunk(const Params& P, const Soa& sp, int64_t* __restrict__ rho,
                                                uint8_t* __restrict__ ev, int64_t evlen, int kb, int nb)
{
    __shared__ unsigned long long win[kWindow];
    __shared__ int ncand;
    const int64_t n = P.cnt->n[kIon];
    const uint32_t step = uint32_t(P.cnt->step);
    const uint64_t kw = sink_threshold(P, kIon);
    int64_t beg, end;
    chunk_range(n, kb, nb, beg, end);
    if (beg >= end) return;

    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) win[k] = 0ull;
    if (threadIdx.x == 0) ncand = 0;
    double f0;
    const int wbase = cell_frac(P, sp.x[beg], f0) - kHalo;
    __syncthreads();
    const double* __restrict__ E = P.E;
    uint32_t* __restrict__ cl = P.cand + beg;   // this block's candidate segment
    uint2* __restrict__ cw = P.cand_w + beg;

    int64_t cur = 0;   // this lane's v_x sum (external circuit)
    for (int64_t i0 = beg; i0 < end; i0 += kAdvBlock) {
        const int64_t i = i0 + threadIdx.x;
        const bool act = i < end;
        bool alive = false, cand = false;
        int jn = 0;
        int64_t an = 0;
        uint2 wcd = make_uint2(0u, 0u);
        double vpush = 0.0;   // v_x after the push, before charge exchange
        if (act) {
            double x = sp.x[i];
            double vx = sp.vx[i];
            const uint32_t id = sp.id[i];
            double f;
            const int j = cell_frac(P, x, f);
            const double Ex = E[j] + f * (E[j + 1] - E[j]);
            vx = vx + P.qmdt_i * Ex;
            x = x + vx * P.dti;
            vpush = vx;
            uint8_t code = kEvNone;
            alive = apply_boundary(P, x, code);
            if (alive) {
                const U4 w = philox10(id, step, 0u, kStreamIonStep, P.key0, P.key1);
                const uint64_t k0 = draw52(w.a, w.b);
                if (k0 >= kw) {
                    alive = false;
                    code = kEvWall;
                } else {
                    cand = k0 < P.kcx;
                }
                wcd = make_uint2(w.c, w.d);
            }
            if (alive) {
                sp.x[i] = x;
                sp.vx[i] = vx;
                double fn;
                jn = cell_frac(P, x, fn);
                an = frac_units(fn);
            }
            if (EV && !cand && int64_t(id) < evlen) ev[id] = code;
        }
        const int64_t hp = wave_append(act && !alive, &P.cnt->nh[kIon]);
        if (hp >= 0) {
            if (hp < P.max_holes) P.holes[kIon][hp] = uint32_t(i);
            else set_err(P, kErrLosses);
        }
        list_candidate(cand, &ncand, cl, cw, uint32_t(i), wcd);
        if (P.circuit && alive) cur += vunits(vpush);
        deposit_wave(P, win, wbase, rho, alive, jn, an);
    }
    if (P.circuit) add_current(P.csum + kCurSlots, cur);
    __syncthreads();
    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) {
        const unsigned long long v = win[k];
        if (v != 0ull) {
            const int node = wbase + k;
            if (node >= 0 && node < P.nn) atomicAdd((unsigned long long*)&rho[node], v);
        }
    }
    // phase 2: this block's charge-exchange candidates
    const int nc = ncand;
    for (int k0 = 0; k0 < nc; k0 += kAdvBlock) {
        const int k = k0 + int(threadIdx.x);
        exchange_one<EV>(P, sp, ev, evlen, step, k < nc, k < nc ? cl[k] : 0u, k < nc ? cw[k] : make_uint2(0u, 0u));
    }
}

// ================================================================ FP32 path
// Cell-relative FP32 state: position = cell + offset (offset in [0,1)), so
// resolution does not degrade along the column; velocities in cells per step
// of the species.  Gather and push run in FP32 against the field scaled to
// cells/step^2 (Ef = q dt^2 E / (m dx)); collision candidates convert to FP64
// and share the FP64 collision code; the field solve stays FP64.

__device__ __forceinline__ int64_t frac_units32(float off)
{
    return int64_t(uint32_t(off * 33554432.0f));   // off * 2^25 is exact in FP32
}

// one FP32 leapfrog step; returns false if the particle left a bounded column
__device__ __forceinline__ bool push32(const Params& P, const float* __restrict__ Ef, int& c, float& off,
                                       float& u, uint8_t& code)
{
    const float e0 = ld32(Ef, uint32_t(c)), e1 = ld32(Ef, uint32_t(c) + 1u);
    u = u + (e0 + off * (e1 - e0));
    off = off + u;
    const float fl = floorf(off);
    c += int(fl);
    off = off - fl;
    if (off >= 1.0f) {
        off = 0.0f;
        c += 1;
    }
    if (!(off >= 0.0f && off < 1.0f)) {   // NaN
        set_err(P, kErrRange);
        off = 0.0f;
    }
    if (P.periodic) {
        if (c >= P.nc) c -= P.nc;
        else if (c < 0) c += P.nc;
        if (c < 0 || c >= P.nc) {
            set_err(P, kErrRange);
            c = 0;
            off = 0.0f;
        }
        return true;
    }
    if (c >= 0 && c < P.nc) return true;
    code = kEvAbsorb;
    return false;
}

template <bool EV>
__device__ __forceinline__ void push_e_chunk(const Params& P, const Soa32& sp, int64_t* __restrict__ rho,
                                             uint8_t* __restrict__ ev, int64_t evlen, int kb, int nb)
{
    __shared__ unsigned long long win[kWindow];
    __shared__ int ncand;
    const int64_t n = P.cnt->n[kElectron];
    const uint32_t step = uint32_t(P.cnt->step);
    const uint64_t kw = sink_threshold(P, kElectron);
    int64_t beg, end;
    chunk_range(n, kb, nb, beg, end);
    if (beg >= end) return;
    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) win[k] = 0ull;
    if (threadIdx.x == 0) ncand = 0;
    const int wbase = sp.cell[beg] - kHalo;
    __syncthreads();
    uint32_t* __restrict__ cl = P.cand + beg;
    uint2* __restrict__ cw = P.cand_w + beg;
    const float* __restrict__ Ef = P.Ef_e;
    int pc = 0;
    float poff = 0.0f, pu = 0.0f;
    uint32_t pid = 0;
    const uint32_t ue = uint32_t(end);
    {
        const uint32_t i = uint32_t(beg) + threadIdx.x;
        if (i < ue) {
            pc = ld32(sp.cell, i);
            poff = ld32(sp.off, i);
            pu = ld32(sp.vx, i);
            pid = ld32(sp.id, i);
        }
    }
    int64_t cur = 0;   // this lane's v_x sum (external circuit)
    for (uint32_t i0 = uint32_t(beg); i0 < ue; i0 += kAdvBlock) {
        const uint32_t i = i0 + threadIdx.x;
        const bool act = i < ue;
        bool alive = false, cand = false;
        int jn = 0;
        int64_t an = 0;
        uint2 wcd = make_uint2(0u, 0u);
        int c = pc;
        float off = poff, u = pu;
        const uint32_t id = pid;
        if (i + kAdvBlock < ue) {
            pc = ld32(sp.cell, i + kAdvBlock);
            poff = ld32(sp.off, i + kAdvBlock);
            pu = ld32(sp.vx, i + kAdvBlock);
            pid = ld32(sp.id, i + kAdvBlock);
        }
        if (act) {
            uint8_t code = kEvNone;
            alive = push32(P, Ef, c, off, u, code);
            if (alive) {
                uint32_t k0, k1;
                loop_keys(P, k0, k1);
                const U4 w = philox10(id, step, 0u, kStreamElectronStep, k0, k1);
                const uint64_t k = draw52(w.a, w.b);
                if (k >= kw) {
                    alive = false;
                    code = kEvWall;
                } else {
                    cand = k < P.kn_e;
                }
                wcd = make_uint2(w.c, w.d);
            }
            if (alive) {
                st32(sp.cell, i, c);
                st32(sp.off, i, off);
                st32(sp.vx, i, u);
                jn = c;
                an = frac_units32(off);
            }
            if (EV && !cand && int64_t(id) < evlen) ev[id] = code;
        }
        const int64_t hp = wave_append(act && !alive, &P.cnt->nh[kElectron]);
        if (hp >= 0) {
            if (hp < P.max_holes) P.holes[kElectron][hp] = i;
            else set_err(P, kErrLosses);
        }
        {
            const uint64_t m = __ballot(cand);
            if (m != 0) {
                const int leader = __ffsll((unsigned long long)m) - 1;
                int base = 0;
                if (lane_id() == leader) base = atomicAdd(&ncand, __popcll((unsigned long long)m));
                base = __shfl(base, leader);
                if (cand) {
                    const uint32_t q = uint32_t(base) + lanes_below(m);
                    st32(cl, q, i);
                    st32(cw, q, wcd);
                }
            }
        }
        if (P.circuit && alive) cur += vunits(double(u) * P.u2v_e);
        deposit_wave(P, win, wbase, rho, alive, jn, an);
    }
    if (P.circuit) add_current(P.csum, cur);
    __syncthreads();
    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) {
        const unsigned long long v = win[k];
        if (v != 0ull) {
            const int node = wbase + k;
            if (node >= 0 && node < P.nn) atomicAdd((unsigned long long*)&rho[node], v);
        }
    }
    const int nc = ncand;
    for (int k0 = 0; k0 < nc; k0 += kAdvBlock) {
        const int k = k0 + int(threadIdx.x);
        collide_one<EV>(P, sp, ev, evlen, step, k < nc, k < nc ? cl[k] : 0u,
                        k < nc ? cw[k] : make_uint2(0u, 0u));
    }
}

template <bool EV>
__device__ __forceinline__ void advance_i_chunk(const Params& P, const Soa32& sp, int64_t* __restrict__ rho,
                                                uint8_t* __restrict__ ev, int64_t evlen, int kb, int nb)
{
    __shared__ unsigned long long win[kWindow];
    __shared__ int ncand;
    const int64_t n = P.cnt->n[kIon];
    const uint32_t step = uint32_t(P.cnt->step);
    const uint64_t kw = sink_threshold(P, kIon);
    int64_t beg, end;
    chunk_range(n, kb, nb, beg, end);
    if (beg >= end) return;
    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) win[k] = 0ull;
    if (threadIdx.x == 0) ncand = 0;
    const int wbase = sp.cell[beg] - kHalo;
    __syncthreads();
    uint32_t* __restrict__ cl = P.cand + beg;   // this block's candidate segment
    uint2* __restrict__ cw = P.cand_w + beg;
    int64_t cur = 0;   // this lane's v_x sum (external circuit)
    for (int64_t i0 = beg; i0 < end; i0 += kAdvBlock) {
        const int64_t i = i0 + threadIdx.x;
        const bool act = i < end;
        bool alive = false, cand = false;
        int jn = 0;
        int64_t an = 0;
        uint2 wcd = make_uint2(0u, 0u);
        float upush = 0.0f;   // v_x after the push, before charge exchange
        if (act) {
            int c = sp.cell[i];
            float off = sp.off[i];
            float u = sp.vx[i];
            const uint32_t id = sp.id[i];
            uint8_t code = kEvNone;
            alive = push32(P, P.Ef_i, c, off, u, code);
            upush = u;
            if (alive) {
                const U4 w = philox10(id, step, 0u, kStreamIonStep, P.key0, P.key1);
                const uint64_t k0 = draw52(w.a, w.b);
                if (k0 >= kw) {
                    alive = false;
                    code = kEvWall;
                } else {
                    cand = k0 < P.kcx;
                }
                wcd = make_uint2(w.c, w.d);
            }
            if (alive) {
                sp.cell[i] = c;
                sp.off[i] = off;
                sp.vx[i] = u;
                jn = c;
                an = frac_units32(off);
            }
            if (EV && !cand && int64_t(id) < evlen) ev[id] = code;
        }
        const int64_t hp = wave_append(act && !alive, &P.cnt->nh[kIon]);
        if (hp >= 0) {
            if (hp < P.max_holes) P.holes[kIon][hp] = uint32_t(i);
            else set_err(P, kErrLosses);
        }
        list_candidate(cand, &ncand, cl, cw, uint32_t(i), wcd);
        if (P.circuit && alive) cur += vunits(double(upush) * P.u2v_i);
        deposit_wave(P, win, wbase, rho, alive, jn, an);
    }
    if (P.circuit) add_current(P.csum + kCurSlots, cur);
    __syncthreads();
    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) {
        const unsigned long long v = win[k];
        if (v != 0ull) {
            const int node = wbase + k;
            if (node >= 0 && node < P.nn) atomicAdd((unsigned long long*)&rho[node], v);
        }
    }
    // phase 2: this block's charge-exchange candidates
    const int nc = ncand;
    for (int k0 = 0; k0 < nc; k0 += kAdvBlock) {
        const int k = k0 + int(threadIdx.x);
        exchange_one<EV>(P, sp, ev, evlen, step, k < nc, k < nc ? cl[k] : 0u, k < nc ? cw[k] : make_uint2(0u, 0u));
    }
}

// FP64 position/velocity -> FP32 cell-relative state
__device__ __forceinline__ void to32(const Params& P, double x, double vx, double vy, double vz, double v2u,
                                     int& c, float& off, float& ux, float& uy, float& uz)
{
    const double s = x * P.inv_dx;
    c = int(s);
    if (c > P.nc - 1) c = P.nc - 1;
    if (c < 0) c = 0;
    off = float(s - double(c));
    if (off >= 1.0f) off = 0.99999994f;
    ux = float(vx * v2u);
    uy = float(vy * v2u);
    uz = float(vz * v2u);
}

template <int S>
__global__ __launch_bounds__(256) void k_load32(Params P, Soa32 sp, int64_t n0, double sig)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n0) return;
    const uint32_t stream = S == kElectron ? kStreamElectronLoad : kStreamIonLoad;
    const U4 w = philox10(uint32_t(k), 0u, 0u, stream, P.key0, P.key1);
    double x = unif52(w.a, w.b) * P.L;
    if (x >= P.L) x = 0.0;
    WordStream ws(uint32_t(k), 0u, stream, P.key0, P.key1);
    double g0, g1, g2;
    normal3(ws, g0, g1, g2);
    const double v2u = 1.0 / (S == kElectron ? P.u2v_e : P.u2v_i);
    int c;
    float off, ux, uy, uz;
    to32(P, x, sig * g0, sig * g1, sig * g2, v2u, c, off, ux, uy, uz);
    sp.cell[k] = c;
    sp.off[k] = off;
    sp.vx[k] = ux;
    sp.vt[k] = make_float2(uy, uz);
    sp.id[k] = uint32_t(k);
}

// leapfrog start in cell units: u -= Ef(x) / 2
__global__ __launch_bounds__(256) void k_halfstep32(Params P, Soa32 sp, int64_t n, int S)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float* Ef = S == kElectron ? P.Ef_e : P.Ef_i;
    const int c = sp.cell[k];
    const float off = sp.off[k];
    const float e0 = Ef[c], e1 = Ef[c + 1];
    sp.vx[k] = sp.vx[k] - 0.5f * (e0 + off * (e1 - e0));
}

// x = (cell + off) dx, v = u dx/dt (caller arrays; any may be null)
__global__ __launch_bounds__(256) void k_to64(Params P, Soa32 src, SoaIO dst, int64_t n, int S)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double u2v = S == kElectron ? P.u2v_e : P.u2v_i;
    if (dst.x) dst.x[k] = (double(src.cell[k]) + double(src.off[k])) * P.dx;
    if (dst.vx) dst.vx[k] = double(src.vx[k]) * u2v;
    if (dst.vy || dst.vz) {
        const float2 t = src.vt[k];
        if (dst.vy) dst.vy[k] = double(t.x) * u2v;
        if (dst.vz) dst.vz[k] = double(t.y) * u2v;
    }
    if (dst.id) dst.id[k] = src.id[k];
}

__global__ __launch_bounds__(256) void k_from64(Params P, SoaIO src, Soa32 dst, int64_t n, int S)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double x = src.x[k];
    if (!(x >= 0.0 && x < P.L)) set_err(P, kErrRange);
    const double v2u = 1.0 / (S == kElectron ? P.u2v_e : P.u2v_i);
    int c;
    float off, ux, uy, uz;
    to32(P, x, src.vx[k], src.vy[k], src.vz[k], v2u, c, off, ux, uy, uz);
    dst.cell[k] = c;
    dst.off[k] = off;
    dst.vx[k] = ux;
    dst.vt[k] = make_float2(uy, uz);
    dst.id[k] = src.id[k];
}

// FP32 field copies scaled to cells per step^2 (with the periodic ghost)
__global__ __launch_bounds__(256) void k_scale_field(Params P)
{
    for (int j = threadIdx.x + blockIdx.x * blockDim.x; j <= P.nn; j += blockDim.x * gridDim.x) {
        const double e = (P.periodic && j == P.nc) ? P.E[0] : (j < P.nn ? P.E[j] : P.E[P.nn - 1]);
        P.Ef_e[j] = float(e * P.efs_e);
        P.Ef_i[j] = float(e * P.efs_i);
    }
}

// ----------------------------------------------------------- block helpers
// Exclusive scan over the block (<= 1024 threads) and the block total: DPP
// wave scans, then wave 0 scans the (<= 16) wave totals.
template <typename T>
__device__ T block_excl_scan(T v, T* sh /* >= 1024/64 + 1 entries */, T& total)
{
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const T incl = wave_incl_scan(v);
    if (lane == 63) sh[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        const T w = lane < nw ? sh[lane] : T(0);
        const T wi = wave_incl_scan(w);
        if (lane < nw) sh[lane] = wi - w;
        if (lane == nw - 1) sh[nw] = wi;
    }
    __syncthreads();
    const T res = sh[wid] + incl - v;
    total = sh[nw];
    __syncthreads();
    return res;
}

// Block total of doubles (the same in every thread, fixed combination order)
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const double w = __ockl_wfred_add_f64(v);
    if (lane_id() == 0) sh[wid] = w;
    __syncthreads();
    if (wid == 0) {
        const double t = __ockl_wfred_add_f64(lane_id() < nw ? sh[lane_id()] : 0.0);
        if (lane_id() == 0) sh[nw] = t;
    }
    __syncthreads();
    const double tot = sh[nw];
    __syncthreads();
    return tot;
}

// -------------------------------------------------------------- field solve
// Poisson's equation on the node grid as Gauss's law: with Q_j the net node
// charge (int64, exact), the half-cell fields obey E_{j+1/2} = E_{j-1/2} +
// fpc Q_j, so E_{j+1/2} = E_{1/2} + fpc T_j with T_j = sum_{k=1..j} Q_k an
// exact integer prefix sum.  E_{1/2} follows from the potential condition:
// bounded sum_j E_{j+1/2} dx = -V, periodic (mean charge removed) sum = 0.
// Node fields: centred average inside, half-cell Gauss at the electrodes.
// This is the same three-point system the Thomas algorithm solves.

// Charge loads of the thread's node segment (nodes j0 .. j0 + seg - 1, seg =
// ceil(nn / threads)), all in flight together: indices clamped into the
// arrays, values outside the segment masked by field_solve.  Split from the
// solve so that a caller can issue other loads while these are in flight.
struct FieldLoads {
    int64_t ri[kMaxSeg], re[kMaxSeg];
};
__device__ __forceinline__ FieldLoads field_load(const Params& P, const int64_t* __restrict__ rho_e,
                                                 const int64_t* __restrict__ rho_i)
{
    FieldLoads fl;
    const int nn = P.nn;
    const int seg = (nn + blockDim.x - 1) / blockDim.x;
    const int j0 = threadIdx.x * seg;
#pragma unroll
    for (int k = 0; k < kMaxSeg; ++k) {
        const int j = j0 + k < nn ? j0 + k : nn - 1;
        fl.ri[k] = rho_i[j];
        fl.re[k] = rho_e[j];
    }
    return fl;
}

// The thread's own node charges Q_j and partial sums, taken from the loads
// as soon as they arrive (a caller that issues more loads after these does
// not make the solve wait for those).
struct FieldPre {
    int64_t q[kMaxSeg];
    int64_t loc;     // sum of own Q_j, j >= 1
    double wsum;     // sum of own (nc - j) Q_j, 1 <= j < nc
};
__device__ __forceinline__ FieldPre field_prepare(const Params& P, const FieldLoads& fl)
{
    FieldPre f;
    const int nn = P.nn, nc = P.nc;
    const int seg = (nn + blockDim.x - 1) / blockDim.x;
    const int j0 = threadIdx.x * seg;
    f.loc = 0;
    f.wsum = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxSeg; ++k) {
        const int j = j0 + k;
        const bool own = k < seg && j < nn;
        const int64_t qk = own ? fl.ri[k] - fl.re[k] : 0;
        f.q[k] = qk;
        f.loc += j >= 1 ? qk : 0;
        f.wsum += (j >= 1 && j < nc) ? double(qk) * double(nc - j) : 0.0;
    }
    return f;
}

__device__ void field_solve(const Params& P, const FieldPre& fp, double* __restrict__ E,
                            double* __restrict__ phi, bool ghost, bool scaled, double V)
{
    // One barrier: each wave posts its charge total and its share of
    // S = sum_{j<nc} T_j = sum_{k=1..nc-1} (nc - k) Q_k; every thread then
    // reads the (<= 16) wave entries itself, in wave order, for its scan
    // offset, the totals and S.  The left neighbour's last half-cell field is
    // E_{1/2} + fpc T_{j0-1}, and T_{j0-1} is the thread's own scan offset, so
    // no field value is exchanged between threads.
    __shared__ int64_t shq[kOneBlock / 64];
    __shared__ double shw[kOneBlock / 64];
    __shared__ double shd[kOneBlock / 64 + 1];
    __shared__ int64_t q0s;
    const int nn = P.nn, nc = P.nc;
    const int seg = (nn + blockDim.x - 1) / blockDim.x;
    const int j0 = threadIdx.x * seg;
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int64_t* q = fp.q;
    const int64_t loc = fp.loc;
    const double wsum = fp.wsum;
    const int64_t incl = wave_incl_scan(loc);
    const double wred = __ockl_wfred_add_f64(wsum);
    if (lane_id() == 63) shq[wid] = incl;
    if (lane_id() == 0) shw[wid] = wred;
    if (threadIdx.x == 0) q0s = q[0];
    __syncthreads();
    int64_t off = incl - loc, qtot_excl0 = 0;
    double S = 0.0;
    for (int w = 0; w < nw; ++w) {
        const int64_t t = shq[w];
        if (w < wid) off += t;
        qtot_excl0 += t;
        S += shw[w];
    }
    const int64_t qall = qtot_excl0 + q0s;   // periodic total charge
    // T_j for own nodes (T_0 = 0; Q_0 excluded)
    int64_t T[kMaxSeg];
    {
        int64_t run = off;
#pragma unroll
        for (int k = 0; k < kMaxSeg; ++k) {
            const int j = j0 + k;
            if (k < seg && j < nn && j >= 1) run += q[k];
            T[k] = run;
        }
    }
    // periodic: T_j - j Q / nc (mean charge removed), whose sum over j < nc
    // is S - Q (nc - 1) / 2
    const double qbar = double(qall) / double(nc);
    const double st = P.periodic ? S - 0.5 * double(qall) * double(nc - 1) : S;
    const double eh0 = P.periodic ? -(P.fpc * (st / double(nc))) : -(V / P.L) - P.fpc * (st / double(nc));
    double Eh[kMaxSeg];
#pragma unroll
    for (int k = 0; k < kMaxSeg; ++k) {
        const int j = j0 + k;
        Eh[k] = eh0 + P.fpc * (P.periodic ? double(T[k]) - double(j) * qbar : double(T[k]));
    }
    // left neighbour of node j0 (> 0): half-cell j0 - 1, T_{j0-1} = off; of
    // node 0 (periodic): the last cell's, T_{nc-1} = the total without Q_0
    const double left0 = j0 == 0
        ? (P.periodic ? eh0 + P.fpc * (double(qtot_excl0) - double(nc - 1) * qbar) : 0.0)
        : eh0 + P.fpc * (P.periodic ? double(off) - double(j0 - 1) * qbar : double(off));
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kMaxSeg; ++k) {
        const int j = j0 + k;
        if (k >= seg || j >= nn) break;
        const double left = k == 0 ? left0 : Eh[k - 1];
        double e;
        if (P.periodic) {
            e = -P.E0 + 0.5 * (left + Eh[k]);
        } else if (j == 0) {
            e = Eh[0] - P.fpc * double(q[0]);
        } else if (j == nc) {
            e = left + P.fpc * double(q[k]);
        } else {
            e = 0.5 * (left + Eh[k]);
        }
        if (!(e - e == 0.0)) bad = true;
        E[j] = e;
        if (ghost && P.periodic && j == 0) E[nc] = e;
        if (scaled) {   // FP32 copies in cells per step^2; entry nn: periodic image or last node
            const float fe = float(e * P.efs_e), fi = float(e * P.efs_i);
            P.Ef_e[j] = fe;
            P.Ef_i[j] = fi;
            if (P.periodic ? j == 0 : j == nn - 1) {
                P.Ef_e[nn] = fe;
                P.Ef_i[nn] = fi;
            }
        }
    }
    if (bad) set_err(P, kErrField);
    if (phi != nullptr) {
        // phi_j = -dx sum_{k<j} E_{k+1/2}
        double ls = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxSeg; ++k)
            if (k < seg && j0 + k < nc) ls += Eh[k];
        double tot;
        double run = block_excl_scan<double>(ls, shd, tot);
#pragma unroll
        for (int k = 0; k < kMaxSeg; ++k) {
            const int j = j0 + k;
            if (k >= seg || j >= nn) break;
            phi[j] = j == 0 ? 0.0 : (!P.periodic && j == nc ? V : -P.dx * run);
            if (j < nc) run += Eh[k];
        }
    }
}

__global__ __launch_bounds__(kOneBlock) void k_field(Params P, const int64_t* rho_e, const int64_t* rho_i,
                                                     double* E, double* phi, int ghost)
{
    if (P.poisson || phi != nullptr || !ghost) {
        field_solve(P, field_prepare(P, field_load(P, rho_e, rho_i)), E, phi, ghost != 0, false,
                    P.circuit ? P.cnt->V : P.V);
    } else {
        const double e0 = P.periodic ? -P.E0 : -((P.circuit ? P.cnt->V : P.V) / P.L);
        for (int j = threadIdx.x; j <= P.nn; j += blockDim.x) E[j] = e0;
    }
}

// ------------------------------------------------------------------ finish
// Single workgroup, once per step:
//  1. field solve E^{n+1} from the advance kernels' charges;
//  2. ionization kinematics (energy sharing of eps - U_iz, isotropic scattered
//     and ejected electrons, Maxwellian ion) from the parent's word stream;
//     the parent's velocity is updated in place, the products' charge is
//     deposited;
//  3. loss holes filled from the array tail (both species);
//  4. products appended in parent-id order (new id = next id + rank);
//  5. counters, clearing of the next charge buffers.
constexpr int kListMax = 2048;    // per-step lists handled in LDS (larger: global scratch)
constexpr int kBirthRegs = kListMax / kOneBlock;

// ionization products of birth b: scattered velocity of the parent, ejected
// electron and new ion velocities (same draw order as every other consumer of
// the (id, step) word stream: split, two directions, three normals)
__device__ __forceinline__ void ionize(const Params& P, const Birth& b, uint32_t step, double vs[3],
                                       double ve[3], double vi[3])
{
    WordStream ws(b.pid, step, kStreamElectronStep, P.key0, P.key1);
    const double us = ws.u();
    const double er = b.eps - P.iz_U;
    const double ej = P.share_equal ? 0.5 * er : P.opb_w * tan(us * atan(er / (2.0 * P.opb_w)));
    const double sc = er - ej;
    double nx, ny, nz, mx, my, mz, g0, g1, g2;
    isotropic(ws, nx, ny, nz);
    isotropic(ws, mx, my, mz);
    normal3(ws, g0, g1, g2);
    const double a = sqrt(sc / P.c_eps);
    const double c = sqrt(ej / P.c_eps);
    vs[0] = a * nx; vs[1] = a * ny; vs[2] = a * nz;
    ve[0] = c * mx; ve[1] = c * my; ve[2] = c * mz;
    vi[0] = P.sig_a * g0; vi[1] = P.sig_a * g1; vi[2] = P.sig_a * g2;
}

template <class St>
__device__ __forceinline__ void deposit_global(const Params& P, const St& st, int64_t* rho, double xk)
{
    int64_t a;
    const int j = key_cell(P, st, xk, a);
    int j1 = j + 1;
    if (P.periodic && j1 == P.nc) j1 = 0;
    atomicAdd((unsigned long long*)&rho[j], (unsigned long long)(kUnit - a));
    atomicAdd((unsigned long long*)&rho[j1], (unsigned long long)a);
}

// ------------------------------------------------------------- pair sink
// Section II keeps the particle number constant: for every ionization of the
// step one electron and one ion, each chosen at random among the live
// particles of its species, leave the column.  Ids stay dense in [0, N): the
// products of ionization r (ranked by parent id) take the slots and ids of
// victims r, so the arrays keep their length and order.  Victim r of a
// species takes the first attempt t = 0, 1, ... whose id, floor(w N / 2^32)
// with w word t mod 4 of the Philox block (r, step, t / 4, victim stream),
// no lower rank has taken.
__device__ __forceinline__ uint32_t victim_draw(const Params& P, int species, uint32_t r, uint32_t step,
                                                uint32_t t, uint64_t n)
{
    const U4 w = philox10(r, step, t >> 2, species == kElectron ? kStreamVictimE : kStreamVictimI, P.key0,
                          P.key1);
    const uint32_t q = t & 3u;
    const uint32_t word = q == 0 ? w.a : (q == 1 ? w.b : (q == 2 ? w.c : w.d));
    return uint32_t((uint64_t(word) * n) >> 32);
}

constexpr uint32_t kVictimTries = 1u << 16;

// removes a particle's CIC charge (the deposit of deposit_global, negated)
template <class St>
__device__ __forceinline__ void undeposit_global(const Params& P, const St& st, int64_t* rho, double xk)
{
    int64_t a;
    const int j = key_cell(P, st, xk, a);
    int j1 = j + 1;
    if (P.periodic && j1 == P.nc) j1 = 0;
    atomicAdd((unsigned long long*)&rho[j], (unsigned long long)(a - kUnit));
    atomicAdd((unsigned long long*)&rho[j1], (unsigned long long)(-a));
}

// Victims of the step's nb ionizations (nb <= kListMax): ids and slots in
// LDS, their charge taken out of rho_e / rho_i before the field solve.
template <class St>
__device__ void pair_victims(const Params& P, const St& se, const St& si, int64_t* rho_e, int64_t* rho_i,
                             int64_t nb, uint32_t step, const int64_t id_range[2], uint32_t (*vid)[kListMax],
                             uint32_t (*vslot)[kListMax])
{
    __shared__ int coll;
    const int tid = threadIdx.x, T = blockDim.x;
    if (tid == 0) coll = 0;
    for (int64_t r = tid; r < nb; r += T)
        for (int s = 0; s < 2; ++s) vid[s][r] = victim_draw(P, s, uint32_t(r), step, 0u, uint64_t(id_range[s]));
    __syncthreads();
    // first attempts that repeat a lower rank's (rare: about nb^2 / 2N per step)
    for (int64_t r = tid; r < nb; r += T)
        for (int s = 0; s < 2; ++s)
            for (int64_t q = 0; q < r; ++q)
                if (vid[s][q] == vid[s][r]) {
                    coll = 1;
                    break;
                }
    __syncthreads();
    // the finish kernels run at least 512 threads: lanes 0 and 64 (two
    // waves) redo the ranks of one species each, in rank order
    if (coll && (tid == 0 || tid == 64)) {
        const int s = tid == 0 ? 0 : 1;
        for (int64_t r = 0; r < nb; ++r)
            for (uint32_t t = 0;; ++t) {
                if (t == kVictimTries) {   // bounded search (nb <= N makes it unreachable in practice)
                    set_err(P, kErrBirths);
                    break;
                }
                const uint32_t id = victim_draw(P, s, uint32_t(r), step, t, uint64_t(id_range[s]));
                bool taken = false;
                for (int64_t q = 0; q < r; ++q) taken = taken || vid[s][q] == id;
                if (!taken) {
                    vid[s][r] = id;
                    break;
                }
            }
    }
    __syncthreads();
    for (int64_t r = tid; r < nb; r += T) {
        for (int s = 0; s < 2; ++s) {
            const St& sp = s == 0 ? se : si;
            const uint32_t slot = P.slot_of[s][vid[s][r]];
            vslot[s][r] = slot;
            undeposit_global(P, sp, s == 0 ? rho_e : rho_i, pos_key(P, sp, slot));
        }
    }
    __threadfence();      // the field loads below read the corrected charges
    __syncthreads();
}

// The finish work of a step falls into two independent halves, run by two
// workgroups of one launch: the field (Poisson solve, external circuit) and
// the particles (ionization kinematics, hole filling, products, emission,
// counters).  Products add an electron and an ion at one position, so the
// field does not depend on them; the only shared data are the charge arrays,
// which the particle half adds the products' charge to -- after the field
// half has loaded them: the field workgroup posts the step index + 1 in
// Counters::field_loaded once every thread holds its charges, and the
// particle workgroup waits for that before its first deposit.  Workgroups are
// dispatched in order and the field half never waits, so the wait ends.  The
// pair sink removes victims' charge before the solve: both halves in one
// workgroup then.
constexpr int kRoleBoth = 0, kRoleField = 1, kRoleParticles = 2;
constexpr uint32_t kLoadedSpinMax = 1u << 22;   // s_sleep rounds before giving up (about 0.2 s)

// The flag orders reads before writes only: the field half's charge loads
// must have returned before the particle half's first add to the same arrays.
// The field half writes nothing before the flag that the particle half
// reads, so neither side needs a device-scope release or acquire (on this
// part the release writes back the XCD's L2 -- much of it dirty with the
// push's particle stores -- and each acquiring poll invalidates it).  The
// field half waits for its own loads by handing their values to an empty asm
// statement, the block barrier waits for every wave, and the flag is a
// relaxed device-scope store, coherent across XCDs.  The particle half polls
// with relaxed device-scope loads; its adds are issued after its barrier,
// which follows the poll that saw the flag.
__device__ __forceinline__ void post_field_loaded(const Params& P, int64_t step_in, const FieldPre* fp)
{
    if (fp != nullptr) {
#pragma unroll
        for (int k = 0; k < kMaxSeg; ++k) asm volatile("" ::"v"(fp->q[k]));
    }
    __syncthreads();   // every thread of the field half holds its charges
    if (threadIdx.x == 0)
        __hip_atomic_store(&P.cnt->field_loaded, step_in + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wait_field_loaded(const Params& P, int64_t step_in)
{
    if (threadIdx.x == 0) {
        for (uint32_t it = 0;; ++it) {
            if (__hip_atomic_load(&P.cnt->field_loaded, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == step_in + 1)
                break;
            if (it == kLoadedSpinMax) {   // never expected: flag the step's field as suspect
                set_err(P, kErrField);
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
    }
    __syncthreads();
}

template <class St>
__device__ __forceinline__ void finish_column(const Params& P, const St& se, const St& si, int64_t* rho_e,
                                              int64_t* rho_i, int64_t* zero_a, int64_t* zero_b, int role)
{
    const bool do_field = role != kRoleParticles;
    const bool do_parts = role != kRoleField;
    __shared__ uint32_t sPid[kListMax];
    __shared__ uint32_t sFlag[2][kListMax / 32];
    __shared__ uint32_t sUpd[kOneBlock / 32];
    __shared__ uint32_t sL1[2][kListMax], sL2[2][kListMax];
    __shared__ unsigned int sC[4];
    const int tid = threadIdx.x;
    const int T = blockDim.x;
    // the step's counters (the same words for every thread) and the charge
    // loads of the field solve go first, together: they depend on nothing
    // else.  The charges are reduced to the thread's partial sums before the
    // loads that wait for the counters are issued.
    Counters* cnt = P.cnt;
    const int64_t n_in[2] = {cnt->n[0], cnt->n[1]};
    const int64_t nh_in[2] = {cnt->nh[0], cnt->nh[1]};
    const int64_t id_in[2] = {cnt->next_id[0], cnt->next_id[1]};
    const int64_t nb_in = cnt->nb;
    const int64_t step_in = cnt->step;
    FieldPre fp;
    const bool loaded = do_field && P.poisson && !P.pair;
    if (loaded) fp = field_prepare(P, field_load(P, rho_e, rho_i));
    if (role == kRoleField) post_field_loaded(P, step_in, loaded ? &fp : nullptr);
    int64_t nb = nb_in < P.max_births ? nb_in : P.max_births;
    int64_t nh[2], Np[2];
    bool lds[2];
    for (int s = 0; s < 2; ++s) {
        nh[s] = nh_in[s] <= P.max_holes ? nh_in[s] : 0;   // overflow already flagged
        Np[s] = n_in[s] - nh[s];
        lds[s] = nh[s] <= kListMax;
    }
    if (P.pair) {
        // victims are listed in LDS, and there must be as many live particles
        if (nb > kListMax || nb > id_in[0] || nb > id_in[1]) {
            if (tid == 0) set_err(P, kErrBirths);
            nb = 0;
        }
    } else if (Np[0] + nb > P.cap || Np[1] + nb > P.cap) {
        if (tid == 0) set_err(P, kErrCapacity);
        nb = 0;
    }
    // one hole and one tail slot per thread: the hole list and the tail
    // particles [Np, N) are loaded here, with the first birth of the thread,
    // so that these loads overlap the field solve
    const bool hfast = nh[0] <= T && nh[1] <= T;
    const bool bfast = nb <= int64_t(kBirthRegs) * T;   // every birth held in registers
    // (unconditional loads from clamped, always valid slots: no branch or
    // merge makes the thread wait for them before the field solve)
    int64_t myh[2] = {0, 0};
    PartRegs<St> tail[2];
    Birth b0;
    if (do_parts) {
        for (int s = 0; s < 2; ++s) {
            const bool own = tid < nh[s];
            myh[s] = P.holes[s][own ? tid : 0];
            tail[s] = load_part(s == 0 ? se : si, uint32_t(own ? Np[s] + tid : 0));
        }
        const int64_t k = tid < nb ? tid : 0;
        b0.pid = P.births[k].pid;
        b0.slot = P.births[k].slot;
        b0.x = P.births[k].x;
        b0.eps = P.births[k].eps;
    }
    if (hfast && do_parts) {
        for (int k = tid; k < 2 * (kListMax / 32); k += T) (&sFlag[0][0])[k] = 0u;
        for (int k = tid; k < kOneBlock / 32; k += T) sUpd[k] = 0u;
    }
    if (tid == 0) sC[0] = sC[1] = sC[2] = sC[3] = 0u;
    // 0. pair sink: victims chosen and their charge removed (the hole lists
    //    are empty in this mode, so their LDS arrays hold the victims)
    if (P.pair) {
        pair_victims(P, se, si, rho_e, rho_i, nb, uint32_t(step_in), id_in, sL1, sL2);
        if (P.poisson) fp = field_prepare(P, field_load(P, rho_e, rho_i));
    }
    // 0b. external circuit (section V): the anode potential of this solve from
    //    the step's conduction current (particles' v_x after their push; ions
    //    from their last subcycle step) and the displacement current of the
    //    gap, backward Euler: V' (1 + a) = V_source + R J + a V, a = R eps0/(L dt)
    double Vf = P.V, Jc = 0.0;
    int64_t vi = 0;
    if (P.circuit && do_field) {
        __shared__ int64_t sCur[2];
        static_assert(kCurSlots == 64, "one slot per lane of wave 0");
        if (tid < 64) {   // wave 0 adds the slots up
            const uint64_t e = __ockl_wfred_add_u64(uint64_t(P.csum[tid]));
            const uint64_t a = __ockl_wfred_add_u64(uint64_t(P.csum[kCurSlots + tid]));
            if (tid == 0) {
                sCur[0] = int64_t(e);
                sCur[1] = int64_t(a);
            }
        }
        __syncthreads();
        const int64_t se = sCur[0], sa = sCur[1];
        vi = step_in % P.ion_subcycle == 0 ? sa : cnt->vsum_i;
        Jc = P.circ_jf * double(vi - se);
        Vf = (P.V + P.circ_R * Jc + P.circ_a * cnt->V) / (1.0 + P.circ_a);
    }
    // 1. field E^{n+1}.  An ionization adds an electron and an ion at the same
    //    position, so the net charge -- and the field -- do not depend on this
    //    step's products: the solve needs only the charges deposited by the
    //    advance kernels and runs first.
    //    FP32 particles also get the field scaled to cells per step^2.
    if (do_field && P.poisson) {
        field_solve(P, fp, P.E, nullptr, true, P.Ef_e != nullptr, Vf);
    } else if (do_field) {
        const double e0 = P.periodic ? -P.E0 : -(Vf / P.L);
        for (int j = tid; j <= P.nn; j += T) {
            P.E[j] = e0;
            if (P.Ef_e != nullptr) {
                P.Ef_e[j] = float(e0 * P.efs_e);
                P.Ef_i[j] = float(e0 * P.efs_i);
            }
        }
    }
    if (role == kRoleField) {
        // the circuit state of this solve; the next charge buffers and the
        // current slots cleared for the next step
        if (tid == 0 && P.circuit) {
            cnt->V = Vf;
            cnt->J = Jc;
            if (step_in % P.ion_subcycle == 0) cnt->vsum_i = vi;
        }
        for (int j = tid; j < P.nn; j += T) {
            if (zero_a) zero_a[j] = 0;
            if (zero_b) zero_b[j] = 0;
        }
        if (P.circuit && tid < kCurSlots) {
            P.csum[tid] = 0;
            if (step_in % P.ion_subcycle == 0) P.csum[kCurSlots + tid] = 0;
        }
        return;
    }
    __syncthreads();   // (orders the LDS clears above against their use)
    const uint32_t step = uint32_t(step_in);

    // 2. births: parent update, products' charge; product velocities kept in
    //    registers (lists longer than kListMax recompute them in step 3)
    double bve[kBirthRegs][3], bvi[kBirthRegs][3], bx[kBirthRegs];
    uint32_t bpid[kBirthRegs];
    bool waited = false;   // particle half: the field half's charges are loaded
#pragma unroll
    for (int m = 0; m < kBirthRegs; ++m) {
        bpid[m] = 0;
        bx[m] = 0.0;
        for (int q = 0; q < 3; ++q) { bve[m][q] = 0.0; bvi[m][q] = 0.0; }
    }
    if (bfast) {
#pragma unroll
        for (int m = 0; m < kBirthRegs; ++m) {
            const int64_t k = tid + int64_t(m) * T;
            if (k < nb) {
                const Birth b = m == 0 ? b0 : P.births[k];
                double vs[3];
                ionize(P, b, step, vs, bve[m], bvi[m]);
                store_v(P, se, b.slot, kElectron, vs[0], vs[1], vs[2]);
                // a parent in the tail: its mover reads the new velocity back
                if (hfast && b.slot >= Np[0] && b.slot < Np[0] + nh[0])
                    atomicOr(&sUpd[(b.slot - Np[0]) >> 5], 1u << ((b.slot - Np[0]) & 31));
                sPid[k] = b.pid;
                bpid[m] = b.pid;
                bx[m] = b.x;
            }
        }
        // the products' charge, once the field half holds this step's charges
        if (role == kRoleParticles && nb > 0) {
            wait_field_loaded(P, step_in);
            waited = true;
        }
#pragma unroll
        for (int m = 0; m < kBirthRegs; ++m) {
            const int64_t k = tid + int64_t(m) * T;
            if (k < nb) {
                deposit_global(P, se, rho_e, bx[m]);
                deposit_global(P, si, rho_i, bx[m]);
            }
        }
    } else {
        if (role == kRoleParticles && nb > 0) {
            wait_field_loaded(P, step_in);
            waited = true;
        }
        for (int64_t k = tid; k < nb; k += T) {
            const Birth b = P.births[k];
            double vs[3], ve[3], vi[3];
            ionize(P, b, step, vs, ve, vi);
            store_v(P, se, b.slot, kElectron, vs[0], vs[1], vs[2]);
            if (hfast && b.slot >= Np[0] && b.slot < Np[0] + nh[0])
                atomicOr(&sUpd[(b.slot - Np[0]) >> 5], 1u << ((b.slot - Np[0]) & 31));
            deposit_global(P, se, rho_e, b.x);
            deposit_global(P, si, rho_i, b.x);
        }
    }
    // 3. hole filling from the tail [Np, N).  One hole per thread: tail holes
    //    are flagged, holes below Np listed; the k-th surviving tail particle
    //    (prefetched) moves to the k-th listed hole.
    if (hfast && (nh[0] > 0 || nh[1] > 0)) {
        for (int s = 0; s < 2; ++s)
            if (tid < nh[s]) {
                const int64_t h = myh[s];
                if (h < Np[s]) sL1[s][atomicAdd(&sC[2 * s], 1u)] = uint32_t(h);
                else if (h < n_in[s]) atomicOr(&sFlag[s][(h - Np[s]) >> 5], 1u << ((h - Np[s]) & 31));
            }
        __syncthreads();
        for (int s = 0; s < 2; ++s) {
            if (tid >= nh[s] || ((sFlag[s][tid >> 5] >> (tid & 31)) & 1u)) continue;
            unsigned int holes_before = __popc(sFlag[s][tid >> 5] & ((1u << (tid & 31)) - 1u));
            for (int w = 0; w < (tid >> 5); ++w) holes_before += __popc(sFlag[s][w]);
            const unsigned int r = unsigned(tid) - holes_before;
            if (r >= sC[2 * s]) continue;   // cannot happen: as many survivors as holes below Np
            const uint32_t dst = sL1[s][r];
            if (s == 0 && ((sUpd[tid >> 5] >> (tid & 31)) & 1u)) move_particle(se, dst, uint32_t(Np[0] + tid));
            else store_part(s == 0 ? se : si, dst, tail[s]);
        }
    } else if (nh[0] > 0 || nh[1] > 0) {   // longer lists: LDS, else global scratch
    for (int s = 0; s < 2; ++s)
        if (lds[s])
            for (int k = tid; k < kListMax / 32; k += T) sFlag[s][k] = 0u;
    __syncthreads();
    for (int s = 0; s < 2; ++s) {
        if (!lds[s] || nh[s] == 0) continue;
        for (int64_t k = tid; k < nh[s]; k += T) {
            const int64_t h = P.holes[s][k];
            if (h >= Np[s]) atomicOr(&sFlag[s][(h - Np[s]) >> 5], 1u << ((h - Np[s]) & 31));
            else sL1[s][atomicAdd(&sC[2 * s], 1u)] = uint32_t(h);
        }
    }
    __syncthreads();
    for (int s = 0; s < 2; ++s) {
        if (!lds[s] || nh[s] == 0) continue;
        for (int64_t k = tid; k < nh[s]; k += T)
            if (!((sFlag[s][k >> 5] >> (k & 31)) & 1u)) sL2[s][atomicAdd(&sC[2 * s + 1], 1u)] = uint32_t(Np[s] + k);
    }
    __syncthreads();
    for (int s = 0; s < 2; ++s) {
        if (!lds[s] || nh[s] == 0) continue;
        const St sp = s == 0 ? se : si;
        for (unsigned int k = tid; k < sC[2 * s]; k += T) move_particle(sp, sL1[s][k], sL2[s][k]);
    }
    // large hole lists: the same algorithm on global scratch, one species at a time
    for (int s = 0; s < 2; ++s) {
        if (lds[s] || nh[s] == 0) continue;
        const St sp = s == 0 ? se : si;
        const int64_t words = (nh[s] + 31) >> 5;
        if (tid == 0) { sC[0] = 0u; sC[1] = 0u; }
        for (int64_t k = tid; k < words; k += T) P.bitmap[k] = 0u;
        __threadfence_block();
        __syncthreads();
        for (int64_t k = tid; k < nh[s]; k += T) {
            const int64_t h = P.holes[s][k];
            if (h >= Np[s]) atomicOr(&P.bitmap[(h - Np[s]) >> 5], 1u << ((h - Np[s]) & 31));
        }
        __threadfence_block();
        __syncthreads();
        uint32_t* L1 = P.lists;
        uint32_t* L2 = P.lists + P.max_holes;
        for (int64_t k = tid; k < nh[s]; k += T) {
            const int64_t h = P.holes[s][k];
            if (h < Np[s]) L1[atomicAdd(&sC[0], 1u)] = uint32_t(h);
            if (!((P.bitmap[k >> 5] >> (k & 31)) & 1u)) L2[atomicAdd(&sC[1], 1u)] = uint32_t(Np[s] + k);
        }
        __threadfence_block();
        __syncthreads();
        for (unsigned int k = tid; k < sC[0]; k += T) move_particle(sp, L1[k], L2[k]);
        __threadfence_block();
        __syncthreads();
    }
    }   // any holes
    __syncthreads();
    // 4. append products at Np + rank (rank of the parent id among this step's)
    if (bfast) {
#pragma unroll
        for (int m = 0; m < kBirthRegs; ++m) {
            const int64_t k = tid + int64_t(m) * T;
            if (k < nb) {
                int64_t r = 0;
                for (int64_t q = 0; q < nb; ++q) r += sPid[q] < bpid[m] ? 1 : 0;
                if (P.pair) {   // into victim r's slots, with its ids
                    put_particle(P, se, sL2[0][r], kElectron, bx[m], bve[m], sL1[0][r]);
                    put_particle(P, si, sL2[1][r], kIon, bx[m], bvi[m], sL1[1][r]);
                } else {
                    put_particle(P, se, Np[0] + r, kElectron, bx[m], bve[m], uint32_t(id_in[0] + r));
                    put_particle(P, si, Np[1] + r, kIon, bx[m], bvi[m], uint32_t(id_in[1] + r));
                }
            }
        }
    } else {
        for (int64_t k = tid; k < nb; k += T) {
            const Birth b = P.births[k];
            double vs[3], ve[3], vi[3];
            ionize(P, b, step, vs, ve, vi);
            int64_t r = 0;
            for (int64_t q = 0; q < nb; ++q) r += P.births[q].pid < b.pid ? 1 : 0;
            if (P.pair) {
                put_particle(P, se, sL2[0][r], kElectron, b.x, ve, sL1[0][r]);
                put_particle(P, si, sL2[1][r], kIon, b.x, vi, sL1[1][r]);
            } else {
                put_particle(P, se, Np[0] + r, kElectron, b.x, ve, uint32_t(id_in[0] + r));
                put_particle(P, si, Np[1] + r, kIon, b.x, vi, uint32_t(id_in[1] + r));
            }
        }
    }
    // 4b. cathode emission (section V): J_e0 dt / (e W) electrons per step, the
    //     fraction carried over; flux-weighted half-Maxwellian at T_c entering
    //     at x = 0, each a uniform fraction of a step in flight; ids after the
    //     products', draws from the new id's own stream
    const int64_t grow = P.pair ? 0 : nb;   // pair sink: products replace the victims
    const double ce = P.emit ? cnt->carry + P.emit_n : 0.0;
    int64_t n_emit = int64_t(floor(ce));
    if (Np[0] + grow + n_emit > P.cap) {
        if (tid == 0) set_err(P, kErrCapacity);
        n_emit = 0;
    }
    for (int64_t r = tid; r < n_emit; r += T) {
        const uint32_t id = uint32_t(id_in[0] + grow + r);
        const U4 w = philox10(id, uint32_t(step_in), 0u, kStreamEmit, P.key0, P.key1);
        double v[3];
        v[0] = P.emit_sig * sqrt(-2.0 * log(unif52(w.a, w.b)));
        double x = v[0] * P.dt * unif52(w.c, w.d);
        if (!(x < P.L)) x = 0.0;
        WordStream ws(id, uint32_t(step_in), kStreamEmit, P.key0, P.key1);
        double g0, g1;
        normal_pair(ws, g0, g1);
        v[1] = P.emit_sig * g0;
        v[2] = P.emit_sig * g1;
        put_particle(P, se, Np[0] + grow + r, kElectron, key_of_x(P, se, x), v, id);
    }
    // 5. counters (no other thread of this kernel reads them) and clearing of
    //    the next charge buffers; nothing here waits for the particle stores.
    //    The particle half writes the step index only after the field half
    //    has read it (and every other counter it reads).
    if (role == kRoleParticles && !waited) wait_field_loaded(P, step_in);
    if (tid == 0) {
        cnt->n[0] = Np[0] + grow + n_emit;
        cnt->n[1] = Np[1] + grow;
        cnt->next_id[0] = id_in[0] + grow + n_emit;
        cnt->next_id[1] = id_in[1] + grow;
        if (id_in[0] + grow + n_emit > 0xFFFFFFFFll || id_in[1] + grow > 0xFFFFFFFFll) set_err(P, kErrIds);
        if (P.emit) cnt->carry = ce - double(n_emit);
        if (P.circuit && role == kRoleBoth) {
            cnt->V = Vf;
            cnt->J = Jc;
            if (step_in % P.ion_subcycle == 0) cnt->vsum_i = vi;
        }
        // ionization tallies of the balanced sink (an ion step consumed the
        // tally since the previous one)
        const int64_t since = (step_in % P.ion_subcycle == 0) ? 0 : cnt->births_since_ion;
        cnt->births_since_ion = since + nb;
        cnt->births_last = nb;
        cnt->nb = 0;
        cnt->nh[0] = 0;
        cnt->nh[1] = 0;
        cnt->step = step_in + 1;
    }
    if (role == kRoleBoth) {
        for (int j = tid; j < P.nn; j += T) {
            if (zero_a) zero_a[j] = 0;
            if (zero_b) zero_b[j] = 0;
        }
        // the current slots start the next step at zero (the ions' on their steps)
        if (P.circuit && tid < kCurSlots) {
            P.csum[tid] = 0;
            if (step_in % P.ion_subcycle == 0) P.csum[kCurSlots + tid] = 0;
        }
    }
}

// -------------------------------------------------------------------- load
// Uniform positions and Maxwellian velocities from the load streams.
template <int S>
__global__ __launch_bounds__(256) void k_load(Params P, Soa sp, int64_t n0, double sig)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n0) return;
    const uint32_t stream = S == kElectron ? kStreamElectronLoad : kStreamIonLoad;
    const U4 w = philox10(uint32_t(k), 0u, 0u, stream, P.key0, P.key1);
    double x = unif52(w.a, w.b) * P.L;
    if (x >= P.L) x = 0.0;
    WordStream ws(uint32_t(k), 0u, stream, P.key0, P.key1);
    double g0, g1, g2;
    normal3(ws, g0, g1, g2);
    sp.x[k] = x;
    sp.vx[k] = sig * g0;
    sp.vt[k] = make_double2(sig * g1, sig * g2);
    sp.id[k] = uint32_t(k);
}

// leapfrog start: vx -= (q dt / 2m) E(x)
__global__ __launch_bounds__(256) void k_halfstep(Params P, Soa sp, int64_t n, double hq)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double f;
    const int j = cell_frac(P, sp.x[k], f);
    const double Ex = P.E[j] + f * (P.E[j + 1] - P.E[j]);
    sp.vx[k] = sp.vx[k] - hq * Ex;
}

// plain per-particle deposit of arbitrary positions (rho cleared beforehand)
__global__ __launch_bounds__(256) void k_deposit(Params P, const double* x, int64_t n, int64_t* rho)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double xv = x[k];
    if (!(xv >= 0.0 && xv < P.L)) {
        set_err(P, kErrRange);
        return;
    }
    double f;
    const int j = cell_frac(P, xv, f);
    const int64_t a = frac_units(f);
    int j1 = j + 1;
    if (P.periodic && j1 == P.nc) j1 = 0;
    atomicAdd((unsigned long long*)&rho[j], (unsigned long long)(kUnit - a));
    atomicAdd((unsigned long long*)&rho[j1], (unsigned long long)a);
}

// deposit of an FP32 store (rho cleared beforehand), same weights as the push
__global__ __launch_bounds__(256) void k_deposit32(Params P, Soa32 sp, int64_t n, int64_t* rho)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int j = sp.cell[k];
    const int64_t a = frac_units32(sp.off[k]);
    int j1 = j + 1;
    if (P.periodic && j1 == P.nc) j1 = 0;
    atomicAdd((unsigned long long*)&rho[j], (unsigned long long)(kUnit - a));
    atomicAdd((unsigned long long*)&rho[j1], (unsigned long long)a);
}

// pair sink: the slot of every id (ids must be a permutation of 0..n-1)
template <class St>
__global__ __launch_bounds__(256) void k_slot_map(Params P, St se, St si)
{
    for (int s = 0; s < 2; ++s) {
        const int64_t n = P.cnt->n[s];
        if (P.cnt->next_id[s] != n) {
            if (blockIdx.x == 0 && threadIdx.x == 0) set_err(P, kErrIds);
            continue;
        }
        const uint32_t* __restrict__ ids = s == 0 ? se.id : si.id;
        for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += int64_t(gridDim.x) * blockDim.x) {
            const uint32_t id = ids[k];
            if (int64_t(id) < n) P.slot_of[s][id] = uint32_t(k);
            else set_err(P, kErrIds);
        }
    }
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// Measurement kernel (stream probe): dst = src over n FP64 elements.  Each
// block walks a contiguous chunk in 256-element tiles with one 8-byte element
// per lane, the access form of the particle kernels, four tiles in flight.
__global__ __launch_bounds__(kAdvBlock) void k_stream_copy(const double* __restrict__ src,
                                                           double* __restrict__ dst, int64_t n)
{
    int64_t beg, end;
    chunk_range(n, int(blockIdx.x), int(gridDim.x), beg, end);
    const uint32_t ue = uint32_t(end);
    uint32_t i = uint32_t(beg) + threadIdx.x;
    for (; i + 3u * kAdvBlock < ue; i += 4u * kAdvBlock) {
        const double a = ld32(src, i), b = ld32(src, i + kAdvBlock), c = ld32(src, i + 2u * kAdvBlock),
                     d = ld32(src, i + 3u * kAdvBlock);
        st32(dst, i, a);
        st32(dst, i + kAdvBlock, b);
        st32(dst, i + 2u * kAdvBlock, c);
        st32(dst, i + 3u * kAdvBlock, d);
    }
    for (; i < ue; i += kAdvBlock) st32(dst, i, ld32(src, i));
}

// caller arrays <-> the interleaved transverse velocity of an FP64 store
__global__ __launch_bounds__(256) void k_vt_split(const double2* __restrict__ vt, double* __restrict__ vy,
                                                  double* __restrict__ vz, int64_t n)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double2 t = vt[k];
    if (vy) vy[k] = t.x;
    if (vz) vz[k] = t.y;
}
__global__ __launch_bounds__(256) void k_vt_join(const double* __restrict__ vy, const double* __restrict__ vz,
                                                 double2* __restrict__ vt, int64_t n)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    vt[k] = make_double2(vy[k], vz[k]);
}

__global__ void k_copy_soa(Soa dst, Soa src, int64_t n)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (dst.x && src.x) dst.x[k] = src.x[k];
    if (dst.vx && src.vx) dst.vx[k] = src.vx[k];
    if (dst.vt && src.vt) dst.vt[k] = src.vt[k];
    if (dst.id && src.id) dst.id[k] = src.id[k];
}

// ----------------------------------------------------------------- moments
// Adds the lanes' values a[q] into out[(first + q) nc + j]: the lanes whose
// cell is the first active lane's are summed across the wave and added once
// (the arrays are sorted by cell, so a wave holds one or two cells), the
// other active lanes add their own.  Integer sums: the result does not
// depend on the grouping.
template <int Q>
__device__ __forceinline__ void cell_sums(int64_t* out, int nc, int first, bool act, int j, const int64_t a[Q])
{
    const uint64_t m = __ballot(act);
    if (m == 0) return;
    const int l1 = __ffsll((unsigned long long)m) - 1;
    const int j1 = __builtin_amdgcn_readlane(j, l1);
    const bool in1 = act && j == j1;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint64_t sum = __ockl_wfred_add_u64(in1 ? uint64_t(a[q]) : 0ull);
        if (lane_id() == l1) atomicAdd((unsigned long long*)&out[(first + q) * nc + j1], (unsigned long long)sum);
        if (act && !in1) atomicAdd((unsigned long long*)&out[(first + q) * nc + j], (unsigned long long)a[q]);
    }
}

template <class St>
__global__ __launch_bounds__(256) void k_moments_e(Params P, St sp, int32_t cpg, int64_t* out)
{
    const int64_t n = P.cnt->n[0];
    const int nc = P.nc;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t k0 = int64_t(blockIdx.x) * blockDim.x; k0 < n; k0 += stride) {
        const int64_t k = k0 + threadIdx.x;
        const bool act = k < n;
        int j = 0, b = 240;
        int64_t a[4] = {0, 0, 0, 0};
        if (act) {
            j = cell_at(P, sp, k);
            double vx, vy, vz;
            load_v(P, sp, uint32_t(k), kElectron, vx, vy, vz);
            const double eps = P.c_eps * ((vx * vx + vy * vy) + vz * vz);
            a[0] = 1;
            a[1] = int64_t(eps * 1048576.0);
            a[2] = int64_t(vx * 1024.0);
            a[3] = int64_t(eps * vx * 16.0);
            b = int(eps * 4.0);
        }
        cell_sums<4>(out, nc, 0, act, j, a);
        if (act && b < 240) atomicAdd((unsigned long long*)&out[7 * nc + (j / cpg) * 240 + b], 1ull);
    }
}

template <class St>
__global__ __launch_bounds__(256) void k_moments_i(Params P, St sp, int64_t* out, int reset)
{
    const int64_t n = P.cnt->n[1];
    const int nc = P.nc;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t k0 = int64_t(blockIdx.x) * blockDim.x; k0 < n; k0 += stride) {
        const int64_t k = k0 + threadIdx.x;
        const bool act = k < n;
        int j = 0;
        int64_t a[2] = {0, 0};
        if (act) {
            j = cell_at(P, sp, k);
            double vx, vy, vz;
            load_v(P, sp, uint32_t(k), kIon, vx, vy, vz);
            a[0] = 1;
            a[1] = int64_t(vx * 1024.0);
        }
        cell_sums<2>(out, nc, 4, act, j, a);
    }
    if (blockIdx.x == 0) {
        for (int j = threadIdx.x; j < nc; j += blockDim.x) {
            out[6 * nc + j] = P.iz[j];
        }
    }
    (void)reset;
}

__global__ void k_reset_iz(Params P)
{
    for (int j = threadIdx.x + blockIdx.x * blockDim.x; j < P.nc; j += blockDim.x * gridDim.x) P.iz[j] = 0;
}

// -------------------------------------------------------------------- sort
// Counting sort by cell (histogram, exclusive scan, scatter).  Blocks take
// the same contiguous chunks as the particle kernels; a chunk of an almost
// sorted array covers few cells, so counts and ranks are kept in an LDS
// window of cells and each (block, cell) reserves its output range with one
// global atomic.  The order inside a cell is arbitrary; nothing downstream
// depends on array order.

// lanes of a wave sharing a cell (up to two distinct cells) add their count
// to the window with one LDS atomic; others add one each.  Out-of-window
// lanes go to the global histogram when `glob` is set.
__device__ __forceinline__ void count_wave(int* cw, int wbase, int32_t* glob, bool act, int c)
{
    bool pend = act;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const uint64_t m = __ballot(pend);
        if (m == 0) return;
        const int leader = __ffsll((unsigned long long)m) - 1;
        const int cr = __builtin_amdgcn_readlane(c, leader);
        const bool mine = pend && c == cr;
        const uint64_t mm = __ballot(mine);
        if (lane_id() == leader) {
            const int li = cr - wbase;
            const int k = __popcll((unsigned long long)mm);
            if (li >= 0 && li < kWindow) atomicAdd(&cw[li], k);
            else if (glob) atomicAdd(&glob[cr], k);
        }
        pend = pend && !mine;
    }
    if (pend) {
        const int li = c - wbase;
        if (li >= 0 && li < kWindow) atomicAdd(&cw[li], 1);
        else if (glob) atomicAdd(&glob[c], 1);
    }
}

template <class St>
__device__ __forceinline__ void sort_count_chunk(const Params& P, const St& sp, int S, int kb, int nb)
{
    __shared__ int cw[kWindow];
    const int64_t n = P.cnt->n[S];
    int64_t beg, end;
    chunk_range(n, kb, nb, beg, end);
    if (beg >= end) return;
    for (int k = threadIdx.x; k < kWindow; k += blockDim.x) cw[k] = 0;
    const int wbase = cell_at(P, sp, beg) - kHalo;
    __syncthreads();
    for (int64_t i0 = beg; i0 < end; i0 += blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const bool act = i < end;
        const int c = act ? cell_at(P, sp, i) : 0;
        count_wave(cw, wbase, P.sort_cnt, act, c);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kWindow; k += blockDim.x) {
        const int v = cw[k];
        const int c = wbase + k;
        if (v != 0 && c >= 0 && c < P.nc) atomicAdd(&P.sort_cnt[c], v);
    }
}

__device__ __forceinline__ void sort_scan_column(const Params& P)
{
    __shared__ int64_t sh[kOneBlock / 64 + 1];
    const int nc = P.nc;
    const int seg = (nc + blockDim.x - 1) / blockDim.x;
    const int j0 = threadIdx.x * seg;
    int64_t loc = 0;
    for (int k = 0; k < seg; ++k)
        if (j0 + k < nc) loc += P.sort_cnt[j0 + k];
    int64_t tot;
    int64_t run = block_excl_scan<int64_t>(loc, sh, tot);
    for (int k = 0; k < seg; ++k) {
        const int j = j0 + k;
        if (j < nc) {
            const int32_t c = P.sort_cnt[j];
            P.sort_off[j] = int32_t(run);
            P.sort_cnt[j] = 0;
            run += c;
        }
    }
}

template <class St>
__device__ __forceinline__ void sort_scatter_chunk(const Params& P, const St& src, const St& dst, int S, int kb,
                                                   int nb)
{
    __shared__ int cw[kWindow];
    __shared__ int bw[kWindow];
    const int64_t n = P.cnt->n[S];
    int64_t beg, end;
    chunk_range(n, kb, nb, beg, end);
    if (beg >= end) return;
    for (int k = threadIdx.x; k < kWindow; k += blockDim.x) cw[k] = 0;
    const int wbase = cell_at(P, src, beg) - kHalo;
    __syncthreads();
    // pass 1: in-window counts of this chunk
    for (int64_t i0 = beg; i0 < end; i0 += blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const bool act = i < end;
        const int c = act ? cell_at(P, src, i) : 0;
        count_wave(cw, wbase, nullptr, act, c);
    }
    __syncthreads();
    // one reservation per (block, cell)
    for (int k = threadIdx.x; k < kWindow; k += blockDim.x) {
        const int v = cw[k];
        if (v != 0) bw[k] = atomicAdd(&P.sort_off[wbase + k], v);
        cw[k] = 0;
    }
    __syncthreads();
    // pass 2: ranks inside the reserved ranges; out-of-window particles take
    // single global slots
    for (int64_t i0 = beg; i0 < end; i0 += blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const bool act = i < end;
        const int c = act ? cell_at(P, src, i) : 0;
        int pos = 0;
        bool pend = act;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const uint64_t m = __ballot(pend);
            if (m == 0) break;
            const int leader = __ffsll((unsigned long long)m) - 1;
            const int cr = __builtin_amdgcn_readlane(c, leader);
            const bool mine = pend && c == cr;
            const uint64_t mm = __ballot(mine);
            int base = 0;
            if (lane_id() == leader) {
                const int li = cr - wbase;
                const int k = __popcll((unsigned long long)mm);
                if (li >= 0 && li < kWindow) base = bw[li] + atomicAdd(&cw[li], k);
                else base = atomicAdd(&P.sort_off[cr], k);
            }
            base = __shfl(base, leader);
            if (mine) pos = base + int(lanes_below(mm));
            pend = pend && !mine;
        }
        if (pend) {
            const int li = c - wbase;
            if (li >= 0 && li < kWindow) pos = bw[li] + atomicAdd(&cw[li], 1);
            else pos = atomicAdd(&P.sort_off[c], 1);
        }
        if (act) {
            copy_particle(dst, pos, src, i);
            if (P.pair) P.slot_of[S][src.id[i]] = uint32_t(pos);
        }
    }
}


// ------------------------------------------------------- single-column kernels
// One column per launch: block b of the grid takes chunk b.
template <bool EV, class St>
__global__ __launch_bounds__(kAdvBlock) void k_push_e(Params P, St sp, int64_t* __restrict__ rho,
                                                     uint8_t* __restrict__ ev, int64_t evlen)
{
    push_e_chunk<EV>(P, sp, rho, ev, evlen, int(blockIdx.x), int(gridDim.x));
}
template <bool EV, class St>
__global__ __launch_bounds__(kAdvBlock) void k_advance_i(Params P, St sp, int64_t* __restrict__ rho,
                                                        uint8_t* __restrict__ ev, int64_t evlen)
{
    advance_i_chunk<EV>(P, sp, rho, ev, evlen, int(blockIdx.x), int(gridDim.x));
}
// Threads is the launch bound (512 or 768 threads: up to 256 or 168 VGPRs,
// no spills; 1024 for fields above 768 kMaxSeg nodes)
template <class St, int Threads>
__global__ __launch_bounds__(Threads) void k_finish(Params P, St se, St si, int64_t* rho_e, int64_t* rho_i,
                                                    int64_t* zero_a, int64_t* zero_b)
{
    finish_column(P, se, si, rho_e, rho_i, zero_a, zero_b,
                  P.pair ? kRoleBoth : (blockIdx.x == 0 ? kRoleField : kRoleParticles));
}
template <class St>
__global__ __launch_bounds__(256) void k_sort_count(Params P, St sp, int S)
{
    sort_count_chunk(P, sp, S, int(blockIdx.x), int(gridDim.x));
}
__global__ __launch_bounds__(kOneBlock) void k_sort_scan(Params P) { sort_scan_column(P); }
template <class St>
__global__ __launch_bounds__(256) void k_sort_scatter(Params P, St src, St dst, int S)
{
    sort_scatter_chunk(P, src, dst, S, int(blockIdx.x), int(gridDim.x));
}

// ------------------------------------------------------------ batched kernels
// Many columns per launch.  Each column's parameters and buffers sit in a
// device table; a launch over particle chunks takes its (column, chunk) from
// an item table ordered by column, and the per-column single-workgroup work
// (field, births, losses, sort scan) runs as one workgroup per column.
// The column table is written by the host between launches and only read by
// the kernels, so it is read through the constant address space: the
// compiler then knows that the pointers it holds address global memory and
// emits global loads and stores for them.  Through a plain pointer they would
// be generic (flat) accesses, which also count against the LDS wait counter,
// so that every LDS wait would wait for the outstanding memory operations too.
typedef const __attribute__((address_space(4))) ColumnDev* ColumnTable;
__device__ __forceinline__ const ColumnDev& column_of(const ColumnDev* cols, int i)
{
    return *(const ColumnDev*)&((ColumnTable)cols)[i];
}
template <class St> __device__ __forceinline__ const St& store_of(const ColumnDev& C, int s, int b);
template <> __device__ __forceinline__ const Soa& store_of<Soa>(const ColumnDev& C, int s, int b)
{
    return C.soa[s][b];
}
template <> __device__ __forceinline__ const Soa32& store_of<Soa32>(const ColumnDev& C, int s, int b)
{
    return C.soa32[s][b];
}

template <class St>
__global__ __launch_bounds__(kAdvBlock) void k_batch_push_e(const ColumnDev* __restrict__ cols,
                                                           const BatchItem* __restrict__ items, BatchStep b)
{
    const BatchItem it = items[blockIdx.x];
    const ColumnDev& C = column_of(cols, it.col);
    push_e_chunk<false>(C.P, store_of<St>(C, kElectron, b.cur[kElectron]), C.rho[kElectron][b.re_new],
                        nullptr, 0, it.k, it.nk);
}
template <class St>
__global__ __launch_bounds__(kAdvBlock) void k_batch_advance_i(const ColumnDev* __restrict__ cols,
                                                              const BatchItem* __restrict__ items, BatchStep b)
{
    const BatchItem it = items[blockIdx.x];
    const ColumnDev& C = column_of(cols, it.col);
    advance_i_chunk<false>(C.P, store_of<St>(C, kIon, b.cur[kIon]), C.rho[kIon][b.ri_use], nullptr, 0, it.k,
                           it.nk);
}
template <class St>
__global__ __launch_bounds__(kOneBlock) void k_batch_finish(const ColumnDev* __restrict__ cols, BatchStep b)
{
    // two workgroups per column (field half, then particle half)
    const ColumnDev& C = column_of(cols, blockIdx.x >> 1);
    finish_column(C.P, store_of<St>(C, kElectron, b.cur[kElectron]), store_of<St>(C, kIon, b.cur[kIon]),
                  C.rho[kElectron][b.re_new], C.rho[kIon][b.ri_use], C.rho[kElectron][b.re_old],
                  b.ri_old >= 0 ? C.rho[kIon][b.ri_old] : nullptr,
                  (blockIdx.x & 1) == 0 ? kRoleField : kRoleParticles);
}
template <class St>
__global__ __launch_bounds__(256) void k_batch_sort_count(const ColumnDev* __restrict__ cols,
                                                         const BatchItem* __restrict__ items, int S, int cur)
{
    const BatchItem it = items[blockIdx.x];
    const ColumnDev& C = column_of(cols, it.col);
    sort_count_chunk(C.P, store_of<St>(C, S, cur), S, it.k, it.nk);
}
__global__ __launch_bounds__(kOneBlock) void k_batch_sort_scan(const ColumnDev* __restrict__ cols)
{
    sort_scan_column(column_of(cols, blockIdx.x).P);
}
template <class St>
__global__ __launch_bounds__(256) void k_batch_sort_scatter(const ColumnDev* __restrict__ cols,
                                                           const BatchItem* __restrict__ items, int S, int cur)
{
    const BatchItem it = items[blockIdx.x];
    const ColumnDev& C = column_of(cols, it.col);
    sort_scatter_chunk(C.P, store_of<St>(C, S, cur), store_of<St>(C, S, 1 - cur), S, it.k, it.nk);
}

}  // namespace pcdev

// ------------------------------------------------------------------ launchers
namespace pclaunch {
using namespace pcdev;

static int grid_for(int64_t n, int block, int maxg)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > maxg) g = maxg;
    return int(g);
}

template <class St>
static hipError_t advance_t(const Params& P, int species, const St& sp, int64_t* rho, uint8_t* ev,
                            int64_t evlen, int grid, hipStream_t st, hipEvent_t t0, hipEvent_t t1)
{
    const bool e = ev != nullptr;
    if (species == kElectron) {
        if (t0) {
            if (e) hipExtLaunchKernelGGL((k_push_e<true, St>), dim3(grid), dim3(kAdvBlock), 0, st, t0, t1, 0, P, sp,
                                         rho, ev, evlen);
            else hipExtLaunchKernelGGL((k_push_e<false, St>), dim3(grid), dim3(kAdvBlock), 0, st, t0, t1, 0, P, sp,
                                       rho, ev, evlen);
        } else {
            if (e) hipLaunchKernelGGL((k_push_e<true, St>), dim3(grid), dim3(kAdvBlock), 0, st, P, sp, rho, ev, evlen);
            else hipLaunchKernelGGL((k_push_e<false, St>), dim3(grid), dim3(kAdvBlock), 0, st, P, sp, rho, ev, evlen);
        }
    } else {
        if (t0) return hipErrorInvalidValue;     // only the electron advance is timed
        if (e)
            hipLaunchKernelGGL((k_advance_i<true, St>), dim3(grid), dim3(kAdvBlock), 0, st, P, sp, rho, ev, evlen);
        else
            hipLaunchKernelGGL((k_advance_i<false, St>), dim3(grid), dim3(kAdvBlock), 0, st, P, sp, rho, ev, evlen);
    }
    return hipGetLastError();
}
hipError_t advance(const Params& P, int species, const Soa& sp, int64_t* rho, uint8_t* ev, int64_t evlen,
                   int grid, hipStream_t st, hipEvent_t t0, hipEvent_t t1)
{
    return advance_t(P, species, sp, rho, ev, evlen, grid, st, t0, t1);
}
hipError_t advance(const Params& P, int species, const Soa32& sp, int64_t* rho, uint8_t* ev, int64_t evlen,
                   int grid, hipStream_t st, hipEvent_t t0, hipEvent_t t1)
{
    return advance_t(P, species, sp, rho, ev, evlen, grid, st, t0, t1);
}

template <class St>
static hipError_t finish_t(const Params& P, const St& se, const St& si, int64_t* rho_e, int64_t* rho_i,
                           int64_t* zero_a, int64_t* zero_b, hipStream_t st)
{
    // eight waves when they cover the field's nodes (kMaxSeg per thread):
    // barriers and block scans get cheaper with fewer waves, while four
    // waves leave too few lanes for the birth and hole lists (measured on a
    // 2000-cell column: 512 threads 27.8, 256 threads 28.5, 1024 threads
    // 28.8 microseconds per step)
    // two workgroups (field half, particle half) except with the pair sink
    const dim3 g(P.pair ? 1 : 2);
    if (P.nn <= 512 * kMaxSeg)
        hipLaunchKernelGGL((k_finish<St, 512>), g, dim3(512), 0, st, P, se, si, rho_e, rho_i, zero_a, zero_b);
    else if (P.nn <= 768 * kMaxSeg)
        hipLaunchKernelGGL((k_finish<St, 768>), g, dim3(768), 0, st, P, se, si, rho_e, rho_i, zero_a, zero_b);
    else
        hipLaunchKernelGGL((k_finish<St, kOneBlock>), g, dim3(kOneBlock), 0, st, P, se, si, rho_e, rho_i,
                           zero_a, zero_b);
    return hipGetLastError();
}
hipError_t finish(const Params& P, const Soa& se, const Soa& si, int64_t* rho_e, int64_t* rho_i,
                  int64_t* zero_a, int64_t* zero_b, hipStream_t st)
{
    return finish_t(P, se, si, rho_e, rho_i, zero_a, zero_b, st);
}
hipError_t finish(const Params& P, const Soa32& se, const Soa32& si, int64_t* rho_e, int64_t* rho_i,
                  int64_t* zero_a, int64_t* zero_b, hipStream_t st)
{
    return finish_t(P, se, si, rho_e, rho_i, zero_a, zero_b, st);
}

// ---- batched launches (ColumnDev table and item tables in device memory)
hipError_t batch_push_e(const ColumnDev* cols, int fp32, const BatchItem* items, int n, const BatchStep& b,
                        hipStream_t st, hipEvent_t t0, hipEvent_t t1)
{
    if (n <= 0) {                     // nothing to launch: an empty timed interval
        if (!t0) return hipSuccess;
        const hipError_t e = hipEventRecord(t0, st);
        return e != hipSuccess ? e : hipEventRecord(t1, st);
    }
    if (t0) {
        if (fp32) hipExtLaunchKernelGGL(k_batch_push_e<Soa32>, dim3(n), dim3(kAdvBlock), 0, st, t0, t1, 0, cols,
                                        items, b);
        else hipExtLaunchKernelGGL(k_batch_push_e<Soa>, dim3(n), dim3(kAdvBlock), 0, st, t0, t1, 0, cols, items, b);
    } else {
        if (fp32) hipLaunchKernelGGL(k_batch_push_e<Soa32>, dim3(n), dim3(kAdvBlock), 0, st, cols, items, b);
        else hipLaunchKernelGGL(k_batch_push_e<Soa>, dim3(n), dim3(kAdvBlock), 0, st, cols, items, b);
    }
    return hipGetLastError();
}
hipError_t batch_advance_i(const ColumnDev* cols, int fp32, const BatchItem* items, int n, const BatchStep& b,
                           hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_batch_advance_i<Soa32>, dim3(n), dim3(kAdvBlock), 0, st, cols, items, b);
    else hipLaunchKernelGGL(k_batch_advance_i<Soa>, dim3(n), dim3(kAdvBlock), 0, st, cols, items, b);
    return hipGetLastError();
}
hipError_t batch_finish(const ColumnDev* cols, int n_cols, int fp32, const BatchStep& b, hipStream_t st)
{
    if (fp32) hipLaunchKernelGGL(k_batch_finish<Soa32>, dim3(2 * n_cols), dim3(kOneBlock), 0, st, cols, b);
    else hipLaunchKernelGGL(k_batch_finish<Soa>, dim3(2 * n_cols), dim3(kOneBlock), 0, st, cols, b);
    return hipGetLastError();
}
template <class St>
static hipError_t batch_sort_t(const ColumnDev* cols, int n_cols, int species, const BatchItem* items, int n,
                               int cur, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_batch_sort_count<St>, dim3(n), dim3(256), 0, st, cols, items, species, cur);
    hipLaunchKernelGGL(k_batch_sort_scan, dim3(n_cols), dim3(kOneBlock), 0, st, cols);
    if (n > 0) hipLaunchKernelGGL(k_batch_sort_scatter<St>, dim3(n), dim3(256), 0, st, cols, items, species, cur);
    return hipGetLastError();
}
hipError_t batch_sort(const ColumnDev* cols, int n_cols, int fp32, int species, const BatchItem* items, int n,
                      int cur, hipStream_t st)
{
    if (fp32) return batch_sort_t<Soa32>(cols, n_cols, species, items, n, cur, st);
    return batch_sort_t<Soa>(cols, n_cols, species, items, n, cur, st);
}

hipError_t field(const Params& P, const int64_t* rho_e, const int64_t* rho_i, double* E, double* phi,
                 int ghost, hipStream_t st)
{
    hipLaunchKernelGGL(k_field, dim3(1), dim3(kOneBlock), 0, st, P, rho_e, rho_i, E, phi, ghost);
    return hipGetLastError();
}

hipError_t scale_field(const Params& P, hipStream_t st)
{
    if (P.Ef_e == nullptr) return hipSuccess;
    hipLaunchKernelGGL(k_scale_field, dim3(32), dim3(256), 0, st, P);
    return hipGetLastError();
}

hipError_t load(const Params& P, int species, const Soa& sp, int64_t n0, double sig, hipStream_t st)
{
    const int g = grid_for(n0, 256, 1 << 30);
    if (n0 == 0) return hipSuccess;
    if (species == kElectron)
        hipLaunchKernelGGL(k_load<kElectron>, dim3(g), dim3(256), 0, st, P, sp, n0, sig);
    else
        hipLaunchKernelGGL(k_load<kIon>, dim3(g), dim3(256), 0, st, P, sp, n0, sig);
    return hipGetLastError();
}

hipError_t load(const Params& P, int species, const Soa32& sp, int64_t n0, double sig, hipStream_t st)
{
    const int g = grid_for(n0, 256, 1 << 30);
    if (n0 == 0) return hipSuccess;
    if (species == kElectron)
        hipLaunchKernelGGL(k_load32<kElectron>, dim3(g), dim3(256), 0, st, P, sp, n0, sig);
    else
        hipLaunchKernelGGL(k_load32<kIon>, dim3(g), dim3(256), 0, st, P, sp, n0, sig);
    return hipGetLastError();
}

hipError_t halfstep(const Params& P, const Soa& sp, int64_t n, double hq, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_halfstep, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, P, sp, n, hq);
    return hipGetLastError();
}

hipError_t halfstep(const Params& P, const Soa32& sp, int species, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_halfstep32, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, P, sp, n, species);
    return hipGetLastError();
}

hipError_t to64(const Params& P, const Soa32& src, const SoaIO& dst, int64_t n, int species, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to64, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, P, src, dst, n, species);
    return hipGetLastError();
}

hipError_t from64(const Params& P, const SoaIO& src, const Soa32& dst, int64_t n, int species, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_from64, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, P, src, dst, n, species);
    return hipGetLastError();
}

template <class St>
static hipError_t slot_map_t(const Params& P, const St& se, const St& si, hipStream_t st)
{
    if (!P.pair) return hipSuccess;
    hipLaunchKernelGGL(k_slot_map<St>, dim3(grid_for(P.cap, 256, 4096)), dim3(256), 0, st, P, se, si);
    return hipGetLastError();
}
hipError_t slot_map(const Params& P, const Soa& se, const Soa& si, hipStream_t st)
{
    return slot_map_t(P, se, si, st);
}
hipError_t slot_map(const Params& P, const Soa32& se, const Soa32& si, hipStream_t st)
{
    return slot_map_t(P, se, si, st);
}
hipError_t fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t deposit(const Params& P, const double* x, int64_t n, int64_t* rho, hipStream_t st)
{
    hipError_t e = fill_i64(rho, P.nn, 0, st);
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(k_deposit, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, P, x, n, rho);
    return hipGetLastError();
}

hipError_t deposit(const Params& P, const Soa32& sp, int64_t n, int64_t* rho, hipStream_t st)
{
    hipError_t e = fill_i64(rho, P.nn, 0, st);
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(k_deposit32, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, P, sp, n, rho);
    return hipGetLastError();
}

hipError_t stream_copy(const double* src, double* dst, int64_t n, int blocks, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(kAdvBlock), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t vt_split(const double2* vt, double* vy, double* vz, int64_t n, hipStream_t st)
{
    if (n == 0 || (!vy && !vz)) return hipSuccess;
    hipLaunchKernelGGL(k_vt_split, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, vt, vy, vz, n);
    return hipGetLastError();
}
hipError_t vt_join(const double* vy, const double* vz, double2* vt, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_vt_join, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, vy, vz, vt, n);
    return hipGetLastError();
}

hipError_t copy_soa(const Soa& dst, const Soa& src, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_soa, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}

template <class St>
static hipError_t moments_t(const Params& P, const St& se, const St& si, int32_t cpg, int reset, int64_t* out,
                            int64_t out_len, hipStream_t st)
{
    hipError_t e = fill_i64(out, out_len, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_moments_e<St>, dim3(1024), dim3(256), 0, st, P, se, cpg, out);
    hipLaunchKernelGGL(k_moments_i<St>, dim3(1024), dim3(256), 0, st, P, si, out, reset);
    if (reset) hipLaunchKernelGGL(k_reset_iz, dim3(64), dim3(256), 0, st, P);
    return hipGetLastError();
}
hipError_t moments(const Params& P, const Soa& se, const Soa& si, int32_t cpg, int reset, int64_t* out,
                   int64_t out_len, hipStream_t st)
{
    return moments_t(P, se, si, cpg, reset, out, out_len, st);
}
hipError_t moments(const Params& P, const Soa32& se, const Soa32& si, int32_t cpg, int reset, int64_t* out,
                   int64_t out_len, hipStream_t st)
{
    return moments_t(P, se, si, cpg, reset, out, out_len, st);
}

template <class St>
static hipError_t sort_t(const Params& P, int species, const St& src, const St& dst, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_sort_count<St>, dim3(grid), dim3(256), 0, st, P, src, species);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kOneBlock), 0, st, P);
    hipLaunchKernelGGL(k_sort_scatter<St>, dim3(grid), dim3(256), 0, st, P, src, dst, species);
    return hipGetLastError();
}
hipError_t sort(const Params& P, int species, const Soa& src, const Soa& dst, int grid, hipStream_t st)
{
    return sort_t(P, species, src, dst, grid, st);
}
hipError_t sort(const Params& P, int species, const Soa32& src, const Soa32& dst, int grid, hipStream_t st)
{
    return sort_t(P, species, src, dst, grid, st);
}

int max_nodes() { return kOneBlock * kMaxSeg; }

}  // namespace pclaunch
