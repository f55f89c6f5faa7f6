// kernels.hip -- gfx950 kernels of the 1D PIC-MCC column step.
//
// Layout: structure-of-arrays FP64 particles (x, vx, vy, vz, id) per species,
// int64 fixed-point node charges, FP64 node field.  One wave64 lane per
// particle; blocks take contiguous chunks of the (periodically cell-sorted)
// particle array so that a block's particles cover a narrow window of nodes,
// which is staged in LDS for the deposit.
#include "device.h"
#include "launch.h"

namespace pcdev {

constexpr int kAdvBlock = 256;   // threads per block of the particle kernels
constexpr int kWindow = 256;     // LDS deposit window (nodes) per block
constexpr int kHalo = 64;        // window starts this many nodes before the chunk
constexpr int kOneBlock = 1024;  // threads of the single-workgroup kernels
constexpr int kMaxSeg = 16;      // nodes per thread in the field solve (n_nodes <= 16384)

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void set_err(const Params& P, uint32_t bits) { atomicOr(&P.cnt->err, bits); }

// ---------------------------------------------------------------- deposit
// add one node contribution: LDS window if inside, else global atomic
__device__ __forceinline__ void add_node(unsigned long long* win, int wbase, int64_t* rho, int node,
                                         int64_t v)
{
    const int li = node - wbase;
    if (li >= 0 && li < kWindow)
        atomicAdd(&win[li], (unsigned long long)v);
    else
        atomicAdd((unsigned long long*)&rho[node], (unsigned long long)v);
}

// Wave-aggregated CIC deposit: lanes sharing a cell are summed first (count
// times 2^32 minus the summed fractions to node j, the summed fractions to
// node j+1), up to two distinct cells per wave; the rest deposit per lane.
__device__ __forceinline__ void deposit_wave(const Params& P, unsigned long long* win, int wbase,
                                             int64_t* rho, bool alive, int j, int64_t a)
{
    bool pend = alive;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const uint64_t m = __ballot(pend);
        if (m == 0) return;
        const int leader = __ffsll((unsigned long long)m) - 1;
        const int jr = __builtin_amdgcn_readlane(j, leader);
        const bool mine = pend && j == jr;
        const uint64_t mm = __ballot(mine);
        const double s = wave_sum(mine ? double(a) : 0.0);
        if (lane_id() == leader) {
            const int64_t sa = int64_t(s);
            const int64_t cntm = int64_t(__popcll((unsigned long long)mm));
            int j1 = jr + 1;
            if (P.periodic && j1 == P.nc) j1 = 0;
            add_node(win, wbase, rho, jr, cntm * kUnit - sa);
            add_node(win, wbase, rho, j1, sa);
        }
        pend = pend && !mine;
    }
    if (pend) {
        int j1 = j + 1;
        if (P.periodic && j1 == P.nc) j1 = 0;
        add_node(win, wbase, rho, j, kUnit - a);
        add_node(win, wbase, rho, j1, a);
    }
}

// append the flagged lanes' values to a global list with one atomic per wave
__device__ __forceinline__ int64_t wave_append(bool flag, int64_t* counter)
{
    const uint64_t m = __ballot(flag);
    if (m == 0) return -1;
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd((unsigned long long*)counter, (unsigned long long)__popcll((unsigned long long)m));
    base = __shfl(base, leader);
    return flag ? int64_t(base) + int64_t(lanes_below(m)) : -1;
}

// ---------------------------------------------------------------- advance
// One species, one step: gather, leapfrog push, boundary, radial sink,
// null-collision MCC, ionization / loss records, fused fixed-point deposit.
template <int S>
__global__ __launch_bounds__(kAdvBlock) void k_advance(Params P, Soa sp, int64_t* __restrict__ rho,
                                                      uint8_t* __restrict__ ev, int64_t evlen)
{
    __shared__ unsigned long long win[kWindow];
    const int64_t n = P.cnt->n[S];
    const uint32_t step = uint32_t(P.cnt->step);
    const int64_t per = ((n + gridDim.x - 1) / gridDim.x + 63) & ~int64_t(63);
    const int64_t beg = int64_t(blockIdx.x) * per;
    const int64_t end = beg + per < n ? beg + per : n;
    if (beg >= end) return;

    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) win[k] = 0ull;
    double f0;
    const int wbase = cell_frac(P, sp.x[beg], f0) - kHalo;
    __syncthreads();

    const double dts = S == kElectron ? P.dt : P.dti;
    const double qmdt = S == kElectron ? P.qmdt_e : P.qmdt_i;
    const double Tw = S == kElectron ? P.T_we : P.T_wi;
    const uint32_t stream = S == kElectron ? kStreamElectronStep : kStreamIonStep;
    const double* __restrict__ E = P.E;

    for (int64_t i0 = beg; i0 < end; i0 += kAdvBlock) {
        const int64_t i = i0 + threadIdx.x;
        const bool act = i < end;
        bool alive = false;
        bool born = false;
        int jn = 0;
        int64_t an = 0;
        uint8_t code = kEvNone;
        uint32_t id = 0;
        double x = 0.0;
        // birth record fields
        double bve0 = 0, bve1 = 0, bve2 = 0, bvi0 = 0, bvi1 = 0, bvi2 = 0;
        if (act) {
            x = sp.x[i];
            double vx = sp.vx[i];
            id = sp.id[i];
            double f;
            const int j = cell_frac(P, x, f);
            const double Ex = E[j] + f * (E[j + 1] - E[j]);
            vx = vx + qmdt * Ex;
            x = x + vx * dts;
            alive = true;
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
            } else if (!(x >= 0.0 && x < P.L)) {
                if (!(x < 0.0 || x >= P.L)) set_err(P, kErrRange);
                alive = false;
                code = kEvAbsorb;
            }
            if (alive) {
                const U4 w = philox10(id, step, 0u, stream, P.key0, P.key1);
                const double u0 = unif52(w.a, w.b);
                const double u1 = unif52(w.c, w.d);
                if (u0 >= Tw) {
                    alive = false;
                    code = kEvWall;
                } else if (S == kElectron && u0 < P.P_null) {
                    double vy = sp.vy[i], vz = sp.vz[i];
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
                    WordStream ws(id, step, stream, P.key0, P.key1);
                    double nx, ny, nz;
                    if (R < c1) {
                        code = kEvElastic;
                        isotropic(ws, nx, ny, nz);
                        const double cosx = ((vx * nx + vy * ny) + vz * nz) / v;
                        const double fac = 1.0 - P.mr2 * (1.0 - cosx);
                        const double vn = v * sqrt(fac);
                        vx = vn * nx;
                        vy = vn * ny;
                        vz = vn * nz;
                    } else if (R < c2) {
                        code = kEvExcite;
                        isotropic(ws, nx, ny, nz);
                        const double vn = sqrt((eps - P.ex_U) / P.c_eps);
                        vx = vn * nx;
                        vy = vn * ny;
                        vz = vn * nz;
                    } else if (R < c3) {
                        code = kEvIonize;
                        const double us = ws.u();
                        const double er = eps - P.iz_U;
                        const double ej =
                            P.share_equal ? 0.5 * er : P.opb_w * tan(us * atan(er / (2.0 * P.opb_w)));
                        const double sc = er - ej;
                        double mx, my, mz, g0, g1, g2;
                        isotropic(ws, nx, ny, nz);
                        isotropic(ws, mx, my, mz);
                        normal3(ws, g0, g1, g2);
                        const double vs = sqrt(sc / P.c_eps);
                        const double ve = sqrt(ej / P.c_eps);
                        vx = vs * nx;
                        vy = vs * ny;
                        vz = vs * nz;
                        bve0 = ve * mx;
                        bve1 = ve * my;
                        bve2 = ve * mz;
                        bvi0 = P.sig_a * g0;
                        bvi1 = P.sig_a * g1;
                        bvi2 = P.sig_a * g2;
                        born = true;
                    } else {
                        code = kEvNull;
                    }
                    sp.vy[i] = vy;
                    sp.vz[i] = vz;
                } else if (S == kIon && u0 < P.P_cx) {
                    double vy = sp.vy[i], vz = sp.vz[i];
                    WordStream ws(id, step, stream, P.key0, P.key1);
                    double g0, g1, g2;
                    normal3(ws, g0, g1, g2);
                    const double ax = P.sig_a * g0, ay = P.sig_a * g1, az = P.sig_a * g2;
                    const double dx = vx - ax, dy = vy - ay, dz = vz - az;
                    const double g = sqrt((dx * dx + dy * dy) + dz * dz);
                    if (g > P.g_cap) set_err(P, kErrGCap);
                    if (u1 * P.g_cap < g) {
                        code = kEvCX;
                        vx = ax;
                        vy = ay;
                        vz = az;
                    } else {
                        code = kEvNull;
                    }
                    sp.vy[i] = vy;
                    sp.vz[i] = vz;
                }
            }
            if (alive) {
                sp.x[i] = x;
                sp.vx[i] = vx;
                double fn;
                jn = cell_frac(P, x, fn);
                an = frac_units(fn);
            }
            if (ev != nullptr && int64_t(id) < evlen) ev[id] = code;
        }
        // losses: slot indices for the compaction
        const int64_t hp = wave_append(act && !alive, &P.cnt->nh[S]);
        if (hp >= 0) {
            if (hp < P.max_holes) P.holes[S][hp] = uint32_t(i);
            else set_err(P, kErrLosses);
        }
        // ionization products
        if (S == kElectron) {
            const int64_t bp = wave_append(born, &P.cnt->nb);
            if (bp >= 0) {
                if (bp < P.max_births) {
                    Birth b;
                    b.pid = id;
                    b.pad = 0;
                    b.x = x;
                    b.ve[0] = bve0; b.ve[1] = bve1; b.ve[2] = bve2;
                    b.vi[0] = bvi0; b.vi[1] = bvi1; b.vi[2] = bvi2;
                    P.births[bp] = b;
                    atomicAdd((unsigned long long*)&P.iz[jn], 1ull);
                } else {
                    set_err(P, kErrBirths);
                }
            }
        }
        deposit_wave(P, win, wbase, rho, alive, jn, an);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kWindow; k += kAdvBlock) {
        const unsigned long long v = win[k];
        if (v != 0ull) {
            const int node = wbase + k;
            if (node >= 0 && node < P.nn) atomicAdd((unsigned long long*)&rho[node], v);
        }
    }
}

// ----------------------------------------------------------- block helpers
template <typename T>
__device__ T block_excl_scan(T v, T* sh /* >= 1024/64 + 1 entries */, T& total)
{
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    T incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    if (lane == 63) sh[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = T(0);
        for (int w = 0; w < nw; ++w) {
            const T t = sh[w];
            sh[w] = acc;
            acc += t;
        }
        sh[nw] = acc;
    }
    __syncthreads();
    const T res = sh[wid] + incl - v;
    total = sh[nw];
    __syncthreads();
    return res;
}

template <typename T>
__device__ T block_sum(T v, T* sh)
{
    T tot;
    (void)block_excl_scan<T>(v, sh, tot);
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
__device__ void field_block(const Params& P, const int64_t* __restrict__ rho_e,
                            const int64_t* __restrict__ rho_i, double* __restrict__ E,
                            double* __restrict__ phi, bool ghost)
{
    __shared__ int64_t shi[kOneBlock / 64 + 1];
    __shared__ double shd[kOneBlock / 64 + 1];
    __shared__ double edge[kOneBlock + 1];
    const int nn = P.nn, nc = P.nc;
    const int seg = (nn + blockDim.x - 1) / blockDim.x;
    const int j0 = threadIdx.x * seg;
    int64_t q[kMaxSeg];
    int64_t loc = 0;
#pragma unroll
    for (int k = 0; k < kMaxSeg; ++k) {
        const int j = j0 + k;
        q[k] = 0;
        if (k < seg && j < nn) {
            q[k] = rho_i[j] - rho_e[j];
            if (j >= 1) loc += q[k];
        }
    }
    int64_t qtot_excl0;
    const int64_t off = block_excl_scan<int64_t>(loc, shi, qtot_excl0);
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
    __shared__ int64_t q0s;
    if (threadIdx.x == 0) q0s = q[0];
    __syncthreads();
    const int64_t qall = qtot_excl0 + q0s;   // periodic total charge
    double Tp[kMaxSeg];
    double lsum = 0.0;
    const double qbar = double(qall) / double(nc);
#pragma unroll
    for (int k = 0; k < kMaxSeg; ++k) {
        const int j = j0 + k;
        Tp[k] = 0.0;
        if (k < seg && j < nc) {
            Tp[k] = P.periodic ? double(T[k]) - double(j) * qbar : double(T[k]);
            lsum += Tp[k];
        }
    }
    const double st = block_sum<double>(lsum, shd);
    const double eh0 = P.periodic ? -(P.fpc * (st / double(nc))) : -(P.V / P.L) - P.fpc * (st / double(nc));
    double Eh[kMaxSeg];
#pragma unroll
    for (int k = 0; k < kMaxSeg; ++k) Eh[k] = eh0 + P.fpc * Tp[k];
    // last half-cell field of each thread, for the left neighbour of node j0
    const int jl = (j0 + seg - 1 < nc - 1) ? j0 + seg - 1 : nc - 1;
    if (j0 < nc) edge[threadIdx.x + 1] = Eh[jl - j0];
    __syncthreads();
    if (threadIdx.x == 0) edge[0] = P.periodic ? edge[(nc - 1) / seg + 1] : 0.0;
    __syncthreads();
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kMaxSeg; ++k) {
        const int j = j0 + k;
        if (k >= seg || j >= nn) break;
        const double left = k == 0 ? edge[threadIdx.x] : Eh[k - 1];
        double e;
        if (P.periodic) {
            const double lft = j == 0 ? edge[0] : left;
            e = -P.E0 + 0.5 * (lft + Eh[k]);
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
            phi[j] = j == 0 ? 0.0 : (!P.periodic && j == nc ? P.V : -P.dx * run);
            if (j < nc) run += Eh[k];
        }
    }
}

__global__ __launch_bounds__(kOneBlock) void k_field(Params P, const int64_t* rho_e, const int64_t* rho_i,
                                                     double* E, double* phi, int ghost)
{
    if (P.poisson || phi != nullptr || !ghost) {
        field_block(P, rho_e, rho_i, E, phi, ghost != 0);
    } else {
        const double e0 = P.periodic ? -P.E0 : -(P.V / P.L);
        for (int j = threadIdx.x; j <= P.nn; j += blockDim.x) E[j] = e0;
    }
}

// ------------------------------------------------------------------ finish
// Single workgroup: fill loss holes from the array tail, append ionization
// products ordered by parent id (new ids = next id + rank), deposit them,
// update counters, solve the field, clear the next charge buffers.
__global__ __launch_bounds__(kOneBlock) void k_finish(Params P, Soa se, Soa si, int64_t* rho_e,
                                                      int64_t* rho_i, int64_t* zero_a, int64_t* zero_b)
{
    __shared__ int64_t sh_n[2];
    __shared__ unsigned int sh_c[2];
    const int tid = threadIdx.x;
    const int T = blockDim.x;
    Counters* cnt = P.cnt;
    for (int s = 0; s < 2; ++s) {
        const Soa sp = s == 0 ? se : si;
        const int64_t N = cnt->n[s];
        int64_t nh = cnt->nh[s];
        if (nh > P.max_holes) nh = 0;   // overflow already flagged; state is invalid
        const int64_t Np = N - nh;
        if (tid == 0) { sh_n[s] = Np; sh_c[0] = 0u; sh_c[1] = 0u; }
        if (nh == 0) continue;
        const int64_t words = (nh + 31) >> 5;
        for (int64_t k = tid; k < words; k += T) P.bitmap[k] = 0u;
        __syncthreads();
        for (int64_t k = tid; k < nh; k += T) {
            const int64_t h = P.holes[s][k];
            if (h >= Np) atomicOr(&P.bitmap[(h - Np) >> 5], 1u << ((h - Np) & 31));
        }
        __syncthreads();
        uint32_t* L1 = P.lists;
        uint32_t* L2 = P.lists + P.max_holes;
        for (int64_t k = tid; k < nh; k += T) {
            const int64_t h = P.holes[s][k];
            if (h < Np) L1[atomicAdd(&sh_c[0], 1u)] = uint32_t(h);
            const int64_t t = Np + k;
            if (!((P.bitmap[k >> 5] >> (k & 31)) & 1u)) L2[atomicAdd(&sh_c[1], 1u)] = uint32_t(t);
        }
        __syncthreads();
        const unsigned int m = sh_c[0];
        for (unsigned int k = tid; k < m; k += T) {
            const uint32_t dst = L1[k], src = L2[k];
            sp.x[dst] = sp.x[src];
            sp.vx[dst] = sp.vx[src];
            sp.vy[dst] = sp.vy[src];
            sp.vz[dst] = sp.vz[src];
            sp.id[dst] = sp.id[src];
        }
        __syncthreads();
        if (tid == 0) { sh_c[0] = 0u; sh_c[1] = 0u; }
        __syncthreads();
    }
    __syncthreads();
    const int64_t ne = sh_n[0], ni = sh_n[1];
    int64_t nb = cnt->nb;
    if (nb > P.max_births) nb = P.max_births;
    if (ne + nb > P.cap || ni + nb > P.cap) {
        if (tid == 0) set_err(P, kErrCapacity);
        nb = 0;
    }
    const int64_t ide = cnt->next_id[0], idi = cnt->next_id[1];
    for (int64_t k = tid; k < nb; k += T) {
        const Birth b = P.births[k];
        int64_t r = 0;
        for (int64_t m = 0; m < nb; ++m) r += P.births[m].pid < b.pid ? 1 : 0;
        const int64_t pe = ne + r, pi = ni + r;
        se.x[pe] = b.x; se.vx[pe] = b.ve[0]; se.vy[pe] = b.ve[1]; se.vz[pe] = b.ve[2];
        se.id[pe] = uint32_t(ide + r);
        si.x[pi] = b.x; si.vx[pi] = b.vi[0]; si.vy[pi] = b.vi[1]; si.vz[pi] = b.vi[2];
        si.id[pi] = uint32_t(idi + r);
        double f;
        const int j = cell_frac(P, b.x, f);
        const int64_t a = frac_units(f);
        int j1 = j + 1;
        if (P.periodic && j1 == P.nc) j1 = 0;
        atomicAdd((unsigned long long*)&rho_e[j], (unsigned long long)(kUnit - a));
        atomicAdd((unsigned long long*)&rho_e[j1], (unsigned long long)a);
        atomicAdd((unsigned long long*)&rho_i[j], (unsigned long long)(kUnit - a));
        atomicAdd((unsigned long long*)&rho_i[j1], (unsigned long long)a);
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        cnt->n[0] = ne + nb;
        cnt->n[1] = ni + nb;
        cnt->next_id[0] = ide + nb;
        cnt->next_id[1] = idi + nb;
        if (ide + nb > 0xFFFFFFFFll || idi + nb > 0xFFFFFFFFll) set_err(P, kErrIds);
        cnt->nb = 0;
        cnt->nh[0] = 0;
        cnt->nh[1] = 0;
    }
    if (P.poisson) {
        field_block(P, rho_e, rho_i, P.E, nullptr, true);
    } else {
        const double e0 = P.periodic ? -P.E0 : -(P.V / P.L);
        for (int j = tid; j <= P.nn; j += T) P.E[j] = e0;
    }
    for (int j = tid; j < P.nn; j += T) {
        if (zero_a) zero_a[j] = 0;
        if (zero_b) zero_b[j] = 0;
    }
    __syncthreads();
    if (tid == 0) cnt->step += 1;
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
    sp.vy[k] = sig * g1;
    sp.vz[k] = sig * g2;
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

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

__global__ void k_copy_soa(Soa dst, Soa src, int64_t n)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (dst.x && src.x) dst.x[k] = src.x[k];
    if (dst.vx && src.vx) dst.vx[k] = src.vx[k];
    if (dst.vy && src.vy) dst.vy[k] = src.vy[k];
    if (dst.vz && src.vz) dst.vz[k] = src.vz[k];
    if (dst.id && src.id) dst.id[k] = src.id[k];
}

// ----------------------------------------------------------------- moments
__global__ __launch_bounds__(256) void k_moments_e(Params P, Soa sp, int32_t cpg, int64_t* out)
{
    const int64_t n = P.cnt->n[0];
    const int nc = P.nc;
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x) {
        double f;
        const int j = cell_frac(P, sp.x[k], f);
        const double vx = sp.vx[k], vy = sp.vy[k], vz = sp.vz[k];
        const double eps = P.c_eps * ((vx * vx + vy * vy) + vz * vz);
        atomicAdd((unsigned long long*)&out[j], 1ull);
        atomicAdd((unsigned long long*)&out[nc + j], (unsigned long long)int64_t(eps * 1048576.0));
        atomicAdd((unsigned long long*)&out[2 * nc + j], (unsigned long long)int64_t(vx * 1024.0));
        atomicAdd((unsigned long long*)&out[3 * nc + j], (unsigned long long)int64_t(eps * vx * 16.0));
        const int b = int(eps * 4.0);
        if (b < 240) atomicAdd((unsigned long long*)&out[7 * nc + (j / cpg) * 240 + b], 1ull);
    }
}

__global__ __launch_bounds__(256) void k_moments_i(Params P, Soa sp, int64_t* out, int reset)
{
    const int64_t n = P.cnt->n[1];
    const int nc = P.nc;
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x) {
        double f;
        const int j = cell_frac(P, sp.x[k], f);
        atomicAdd((unsigned long long*)&out[4 * nc + j], 1ull);
        atomicAdd((unsigned long long*)&out[5 * nc + j], (unsigned long long)int64_t(sp.vx[k] * 1024.0));
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
// Counting sort by cell: histogram, exclusive scan, scatter.  The order inside
// a cell is arbitrary; nothing downstream depends on array order.
__global__ __launch_bounds__(256) void k_sort_count(Params P, Soa sp, int S)
{
    const int64_t n = P.cnt->n[S];
    for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x; i0 < n; i0 += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const bool act = i < n;
        int c = 0;
        if (act) {
            double f;
            c = cell_frac(P, sp.x[i], f);
        }
        bool pend = act;
        for (int it = 0; it < 2; ++it) {
            const uint64_t m = __ballot(pend);
            if (m == 0) break;
            const int leader = __ffsll((unsigned long long)m) - 1;
            const int cr = __builtin_amdgcn_readlane(c, leader);
            const bool mine = pend && c == cr;
            const uint64_t mm = __ballot(mine);
            if (lane_id() == leader) atomicAdd(&P.sort_cnt[cr], __popcll((unsigned long long)mm));
            pend = pend && !mine;
        }
        if (pend) atomicAdd(&P.sort_cnt[c], 1);
    }
}

__global__ __launch_bounds__(kOneBlock) void k_sort_scan(Params P)
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

__global__ __launch_bounds__(256) void k_sort_scatter(Params P, Soa src, Soa dst, int S)
{
    const int64_t n = P.cnt->n[S];
    for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x; i0 < n; i0 += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const bool act = i < n;
        int c = 0;
        if (act) {
            double f;
            c = cell_frac(P, src.x[i], f);
        }
        int64_t pos = -1;
        bool pend = act;
        for (int it = 0; it < 2; ++it) {
            const uint64_t m = __ballot(pend);
            if (m == 0) break;
            const int leader = __ffsll((unsigned long long)m) - 1;
            const int cr = __builtin_amdgcn_readlane(c, leader);
            const bool mine = pend && c == cr;
            const uint64_t mm = __ballot(mine);
            int base = 0;
            if (lane_id() == leader) base = atomicAdd(&P.sort_off[cr], __popcll((unsigned long long)mm));
            base = __shfl(base, leader);
            if (mine) pos = base + int(lanes_below(mm));
            pend = pend && !mine;
        }
        if (pend) pos = atomicAdd(&P.sort_off[c], 1);
        if (act) {
            dst.x[pos] = src.x[i];
            dst.vx[pos] = src.vx[i];
            dst.vy[pos] = src.vy[i];
            dst.vz[pos] = src.vz[i];
            dst.id[pos] = src.id[i];
        }
    }
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

hipError_t advance(const Params& P, int species, const Soa& sp, int64_t* rho, uint8_t* ev, int64_t evlen,
                   int grid, hipStream_t st)
{
    if (species == kElectron)
        hipLaunchKernelGGL(k_advance<kElectron>, dim3(grid), dim3(kAdvBlock), 0, st, P, sp, rho, ev, evlen);
    else
        hipLaunchKernelGGL(k_advance<kIon>, dim3(grid), dim3(kAdvBlock), 0, st, P, sp, rho, ev, evlen);
    return hipGetLastError();
}

hipError_t finish(const Params& P, const Soa& se, const Soa& si, int64_t* rho_e, int64_t* rho_i,
                  int64_t* zero_a, int64_t* zero_b, hipStream_t st)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kOneBlock), 0, st, P, se, si, rho_e, rho_i, zero_a, zero_b);
    return hipGetLastError();
}

hipError_t field(const Params& P, const int64_t* rho_e, const int64_t* rho_i, double* E, double* phi,
                 int ghost, hipStream_t st)
{
    hipLaunchKernelGGL(k_field, dim3(1), dim3(kOneBlock), 0, st, P, rho_e, rho_i, E, phi, ghost);
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

hipError_t halfstep(const Params& P, const Soa& sp, int64_t n, double hq, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_halfstep, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, P, sp, n, hq);
    return hipGetLastError();
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

hipError_t copy_soa(const Soa& dst, const Soa& src, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_soa, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}

hipError_t moments(const Params& P, const Soa& se, const Soa& si, int32_t cpg, int reset, int64_t* out,
                   int64_t out_len, hipStream_t st)
{
    hipError_t e = fill_i64(out, out_len, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_moments_e, dim3(1024), dim3(256), 0, st, P, se, cpg, out);
    hipLaunchKernelGGL(k_moments_i, dim3(1024), dim3(256), 0, st, P, si, out, reset);
    if (reset) hipLaunchKernelGGL(k_reset_iz, dim3(64), dim3(256), 0, st, P);
    return hipGetLastError();
}

hipError_t sort(const Params& P, int species, const Soa& src, const Soa& dst, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_sort_count, dim3(grid), dim3(256), 0, st, P, src, species);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kOneBlock), 0, st, P);
    hipLaunchKernelGGL(k_sort_scatter, dim3(grid), dim3(256), 0, st, P, src, dst, species);
    return hipGetLastError();
}

int max_nodes() { return kOneBlock * kMaxSeg; }

}  // namespace pclaunch
