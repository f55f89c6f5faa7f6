// fluid.hip -- gfx950 kernels of the batched quasi-neutral fluid column
// (section IV of the paper, eqs. (3)-(17)).
//
// Per time step and column (many columns per launch, one workgroup each):
//   k_fluid_faces  temperatures, transport coefficients from the table
//                  (linear interpolation in T), face states, the total flux
//                  Gamma_T fixed by the imposed mean field, the field of
//                  eq. (17), the closure fluxes of eqs. (12)-(13) -- or the
//                  normalised inputs of the closure network (the network then
//                  runs on the matrix cores, mlp.hip), which either gives the
//                  fluxes or multipliers of the tabulated coefficients used
//                  by eqs. (12)-(13) on the next step
//   k_fluid_solve  sources (ionisation minus radial loss, Joule heating minus
//                  collisional loss), backward-Euler diffusion of density and
//                  of energy density as two cyclic tridiagonal systems in
//                  FP64, solved by cyclic reduction in LDS
//   k_fluid_step   both in one workgroup per column, for the closures whose
//                  fluxes the face pass computes (table, multipliers); the
//                  network flux closure runs faces, network and solve apart
// State and face arrays are FP32; the tridiagonal systems are FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/pc_fluid.h"
#include "../../include/pc_mlp.h"

namespace pcfluid {

constexpr int kFaceBlock = 1024;   // 16 waves per column: the face loop is latency-bound
constexpr int kSolveBlock = 1024;
constexpr int kMaxCells = 4096;
constexpr int kCols = 6;   // table columns
constexpr int kMaxTableRows = 1024;   // the table is staged in LDS by both kernels (24 KB)
constexpr int kFacesPerThread = kMaxCells / kFaceBlock;
// LDS rows of the tridiagonal systems: element j at pad(j) = j + j / 32, one
// spare double per 32, so that the reduction's strided accesses (equations
// 2s apart at level s) spread over the banks instead of piling onto a few
constexpr int kPadCells = kMaxCells + kMaxCells / 32;
__device__ __forceinline__ int pad(int j) { return j + (j >> 5); }

struct ColDev {
    double L, Ngas, E0, nu_w, muiN;
};

// closure kinds
constexpr int kTable = 0, kNetFlux = 1, kNetMult = 2;
constexpr float kMultMin = 0.25f, kMultMax = 4.0f;

struct Globals {
    int32_t N, K, mlp, have_m;   // closure kind; have_m: y holds multipliers of this state's past
    float T_min, T_step, n_floor, dt;
    const float* table;        // [K][6]
    const ColDev* cols;
    float *n, *w;              // [col][N]
    float *gam, *H, *E, *Da, *kap, *dn, *dT;   // faces [col][N], face j between cells j and j+1
    float* x;                  // closure-network inputs [col][N][5]
    const float* y;            // closure-network outputs [col][N][2] (fluxes or multipliers)
    float norm[14];            // inputs (x - off) * scale (5 + 5), outputs y * scale + off (2 + 2)
};

// coefficient row at T (clamped) and its slope
struct Coef {
    float v[kCols];
    float s[kCols];
};

// tab: the workgroup's LDS copy of the table (stage_table)
__device__ __forceinline__ Coef interp(const Globals& G, const float* tab, float T)
{
    const float Tmax = G.T_min + float(G.K - 1) * G.T_step;
    const float Tc = fminf(fmaxf(T, G.T_min), Tmax);
    const float u = (Tc - G.T_min) / G.T_step;
    int k = int(floorf(u));
    if (k > G.K - 2) k = G.K - 2;
    if (k < 0) k = 0;
    const float f = u - float(k);
    Coef c;
    const float* lo = tab + k * kCols;
    const float* hi = lo + kCols;
#pragma unroll
    for (int q = 0; q < kCols; ++q) {
        const float d = hi[q] - lo[q];
        c.v[q] = lo[q] + f * d;
        c.s[q] = d / G.T_step;
    }
    return c;
}

// the table into LDS: a face needs three interpolations, each a dependent
// gather of twelve coefficients
__device__ __forceinline__ void stage_table(const Globals& G, float* tab)
{
    for (int k = threadIdx.x; k < G.K * kCols; k += blockDim.x) tab[k] = G.table[k];
    __syncthreads();
}

__device__ __forceinline__ double block_sum_d(double v, double* sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < int(blockDim.x >> 6); ++k) t += sh[k];   // fixed order
    return t;
}

// face quantities of face j (between cells j and j+1) of one column
struct FaceQ {
    float nf, Tf, dn, dT, A, B, mue, De, mueps, Deps, dDe, dDeps;
};

// multipliers of face j (m_D, m_eps): the network's last answer, clamped; 1 before it
__device__ __forceinline__ void face_multipliers(const Globals& G, int64_t f, float& mD, float& mE)
{
    mD = mE = 1.0f;
    if (G.mlp == kNetMult && G.have_m) {
        mD = fminf(fmaxf(G.y[f * 2] * G.norm[10] + G.norm[12], kMultMin), kMultMax);
        mE = fminf(fmaxf(G.y[f * 2 + 1] * G.norm[11] + G.norm[13], kMultMin), kMultMax);
    }
}

__device__ __forceinline__ FaceQ face(const Globals& G, const float* tab, const ColDev& C, const float* n,
                                      const float* w, int j, float mD, float mE)
{
    const int N = G.N;
    const int jr = (j + 1) & (N - 1);
    const float Ng = float(C.Ngas);
    const float dx = float(C.L / double(N));
    const float n0 = n[j], n1 = n[jr];
    const float T0 = w[j] / (1.5f * n0), T1 = w[jr] / (1.5f * n1);
    const Coef c0 = interp(G, tab, T0), c1 = interp(G, tab, T1);
    const float Phi0 = n0 * (c0.v[1] / Ng) / (c0.v[0] / Ng);
    const float Phi1 = n1 * (c1.v[1] / Ng) / (c1.v[0] / Ng);
    FaceQ q;
    q.nf = 0.5f * (n0 + n1);
    q.Tf = 0.5f * (T0 + T1);
    q.dn = (n1 - n0) / dx;
    q.dT = (T1 - T0) / dx;
    const Coef cf = interp(G, tab, q.Tf);
    q.mue = cf.v[0] / Ng;
    q.De = mD * (cf.v[1] / Ng);
    q.mueps = mE * (cf.v[2] / Ng);
    q.Deps = mE * (cf.v[3] / Ng);
    q.dDe = mD * (cf.s[1] / Ng);
    q.dDeps = mE * (cf.s[3] / Ng);
    const float mui = float(C.muiN) / Ng;
    q.A = mD * ((Phi1 - Phi0) / (dx * q.nf));
    q.B = 1.0f / (q.nf * (q.mue + mui));
    return q;
}

// the values of one face that the solve uses
struct FaceOut {
    float E, Da, kap, dn, dT, gam, H;
};

// outputs of face f from its quantities q and the column's total flux
// Gamma_T: E, the closure fluxes Gamma and H (table and multiplier closures)
// and the network inputs (network closures) are stored; D_a, kappa, dn/dx and
// dT/dx only when the solve runs as a kernel of its own (store_solver)
__device__ __forceinline__ FaceOut face_out(const Globals& G, const FaceQ& q, float GT, float mui, int64_t f,
                                            bool store_solver)
{
    FaceOut r;
    r.E = -q.A + GT * q.B;
    r.Da = mui * q.De / q.mue;
    const float beta = 1.5f * q.Tf * q.mueps;
    const float Gc = 1.5f * q.Tf * q.Deps;
    const float dG = 1.5f * q.Deps + 1.5f * q.Tf * q.dDeps;
    r.kap = q.nf * (dG - beta * q.dDe / q.mue);
    r.dn = q.dn;
    r.dT = q.dT;
    r.gam = 0.0f;
    r.H = 0.0f;
    G.E[f] = r.E;
    if (store_solver) {
        G.Da[f] = r.Da;
        G.kap[f] = r.kap;
        G.dn[f] = q.dn;
        G.dT[f] = q.dT;
    }
    if (G.mlp != kTable) {
        const float x[5] = {q.nf, 1.5f * q.Tf, r.E, q.dn, 1.5f * q.dT};
        float* xo = G.x + f * 5;
#pragma unroll
        for (int k = 0; k < 5; ++k) xo[k] = (x[k] - G.norm[k]) * G.norm[5 + k];
    }
    if (G.mlp != kNetFlux) {
        const float eta = q.nf * (mui / q.mue) * q.dDe;
        const float chi = Gc - beta * q.De / q.mue;
        r.gam = -r.Da * q.dn - eta * q.dT - q.mue / (q.mue + mui) * GT;
        r.H = -chi * q.dn - r.kap * q.dT - beta / (q.mue + mui) * GT;
        G.gam[f] = r.gam;
        G.H[f] = r.H;
    }
    return r;
}

// the faces j = tid + r * kFaceBlock of this workgroup's column, in two
// passes (the column sums of A and B fix Gamma_T first); each face is
// evaluated once and kept in registers between the passes
__device__ __forceinline__ void faces_column(const Globals& G, const ColDev& C, const float* tab, double* sh,
                                             FaceOut (&fo)[kFacesPerThread], bool store_solver)
{
    const int N = G.N;
    const int64_t o = int64_t(blockIdx.x) * N;
    const float* n = G.n + o;
    const float* w = G.w + o;
    FaceQ qs[kFacesPerThread];
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int r = 0; r < kFacesPerThread; ++r) {
        const int j = threadIdx.x + r * kFaceBlock;
        if (j < N) {
            float mD, mE;
            face_multipliers(G, o + j, mD, mE);
            qs[r] = face(G, tab, C, n, w, j, mD, mE);
            sa += double(qs[r].A);
            sb += double(qs[r].B);
        }
    }
    const double SA = block_sum_d(sa, sh);
    const double SB = block_sum_d(sb, sh);
    const float GT = float((C.E0 + SA / N) / (SB / N));
    const float mui = float(C.muiN / C.Ngas);
#pragma unroll
    for (int r = 0; r < kFacesPerThread; ++r) {
        const int j = threadIdx.x + r * kFaceBlock;
        if (j < N) fo[r] = face_out(G, qs[r], GT, mui, o + j, store_solver);
    }
}

__global__ __launch_bounds__(kFaceBlock) void k_fluid_faces(Globals G)
{
    __shared__ double sh[kFaceBlock / 64];
    __shared__ float tab[kMaxTableRows * kCols];
    const ColDev C = G.cols[blockIdx.x];
    stage_table(G, tab);
    FaceOut fo[kFacesPerThread];
    faces_column(G, C, tab, sh, fo, true);
}

// ---- cyclic reduction for a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j,
// indices mod N, N a power of two; in place in LDS (row j at pad(j)),
// solution left in d.
// Level s (1, 2, ..., N/2) eliminates x_{j-s}, x_{j+s} from the equations
// j = 0 mod 2s using equations j -+ s; the last level leaves one equation in
// x_0 alone; back substitution then recovers j = s mod 2s from j -+ s.
// Levels that update more than 64 equations run on the whole workgroup, one
// block barrier each; the rest, down to x_0 and back, on wave 0 alone: the
// LDS operations of one wave complete in issue order, so those levels need
// only compiler ordering.  Every equation sees the same arithmetic in the
// same order either way.
__device__ __forceinline__ void lds_wave_order() { asm volatile("" ::: "memory"); }

// 1/b for the reduction's pivots (diagonally dominant rows: positive, of
// order 1 to r): the hardware estimate refined by two Newton-Raphson steps,
// y <- y + y (1 - b y), to within a rounding of the quotient; about half the
// instructions of a correctly rounded division on the reduction's chain
__device__ __forceinline__ double recip(double b)
{
    double y = __builtin_amdgcn_rcp(b);
    y = fma(fma(-b, y, 1.0), y, y);
    y = fma(fma(-b, y, 1.0), y, y);
    return y;
}

__device__ __forceinline__ void cr_eliminate(double* a, double* b, double* c, double* d, int N, int s, int j0)
{
    const int j = pad(j0), jm = pad((j0 - s) & (N - 1)), jp = pad((j0 + s) & (N - 1));
    const double al = -a[j] * recip(b[jm]);
    const double ga = -c[j] * recip(b[jp]);
    const double na = al * a[jm];
    const double nc = ga * c[jp];
    const double nb = b[j] + al * c[jm] + ga * a[jp];
    const double nd = d[j] + al * d[jm] + ga * d[jp];
    a[j] = na;
    b[j] = nb;
    c[j] = nc;
    d[j] = nd;
}

__device__ __forceinline__ void cr_substitute(const double* a, const double* b, const double* c, double* d, int N,
                                              int s, int j0)
{
    const int j = pad(j0), jm = pad((j0 - s) & (N - 1)), jp = pad((j0 + s) & (N - 1));
    d[j] = (d[j] - a[j] * d[jm] - c[j] * d[jp]) * recip(b[j]);
}

__device__ void cyclic_reduce(double* a, double* b, double* c, double* d, int N)
{
    int s = 1;
    for (; s < N && N / (2 * s) > 64; s <<= 1) {
        __syncthreads();
        for (int j = threadIdx.x * 2 * s; j < N; j += blockDim.x * 2 * s) cr_eliminate(a, b, c, d, N, s, j);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        for (int t = s; t < N; t <<= 1) {
            const int j = threadIdx.x * 2 * t;
            if (j < N) cr_eliminate(a, b, c, d, N, t, j);
            lds_wave_order();
        }
        if (threadIdx.x == 0) d[0] = d[0] / (a[0] + b[0] + c[0]);   // x_{-N} = x_N = x_0
        lds_wave_order();
        for (int t = N >> 1; t >= s; t >>= 1) {
            const int j = t + threadIdx.x * 2 * t;
            if (j < N) cr_substitute(a, b, c, d, N, t, j);
            lds_wave_order();
        }
    }
    for (int t = s >> 1; t >= 1; t >>= 1) {
        __syncthreads();
        for (int j = t + threadIdx.x * 2 * t; j < N; j += blockDim.x * 2 * t) cr_substitute(a, b, c, d, N, t, j);
    }
    __syncthreads();
}

constexpr int kRows = kMaxCells / kSolveBlock;
static_assert(kRows == kFacesPerThread, "a thread's cells are its faces' left cells");

// explicit parts of cell j (sources, the closure fluxes' divergence): the
// density row at pj and, returned, the energy right-hand side; faces p = j
// (right of the cell) and m = j - 1
__device__ __forceinline__ double setup_cell(const Globals& G, const ColDev& C, const float* tab, double r,
                                             double dt, double dx, float nj, float wj, float gp, float gm,
                                             float hp, float hm, float Ep, float Em, float Dap, float Dam, float dnp,
                                             float dnm, float Kpf, float Kmf, float dTp, float dTm, int pj,
                                             double* A, double* B, double* Cc, double* D)
{
    const float Ng = float(C.Ngas);
    const Coef cc = interp(G, tab, wj / (1.5f * nj));
    const float Sn = nj * (Ng * cc.v[4] - float(C.nu_w));
    const float P = -0.5f * (gm * Em + gp * Ep);
    const float Sw = P - nj * (Ng * cc.v[5]);
    const double Dp = Dap, Dm = Dam;
    const double gep = double(gp) + Dp * double(dnp);
    const double gem = double(gm) + Dm * double(dnm);
    A[pj] = -r * Dm;
    B[pj] = 1.0 + r * (Dm + Dp);
    Cc[pj] = -r * Dp;
    D[pj] = double(nj) + dt * double(Sn) - dt / dx * (gep - gem);
    const double Kp = Kpf, Km = Kmf;
    const double hep = double(hp) + Kp * double(dTp);
    const double hem = double(hm) + Km * double(dTm);
    return double(wj) + dt * double(Sw) - dt / dx * (hep - hem);
}

// the density solve, then the energy-density system with T' = w' / (1.5 n')
// and its solve; Kp, Km: kappa of each own cell's right and left faces
__device__ __forceinline__ void solve_tail(const Globals& G, double* A, double* B, double* Cc, double* D,
                                           const double (&rhs_w)[kRows], const float (&Kp)[kRows],
                                           const float (&Km)[kRows], double r)
{
    const int N = G.N;
    const int64_t o = int64_t(blockIdx.x) * N;
    float* n = G.n + o;
    float* w = G.w + o;
    cyclic_reduce(A, B, Cc, D, N);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = threadIdx.x + k * kSolveBlock;
        if (j < N) n[j] = fmaxf(float(D[pad(j)]), G.n_floor);
    }
    __syncthreads();   // new densities visible to the whole workgroup
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = threadIdx.x + k * kSolveBlock;
        if (j < N) {
            const int jm = (j - 1) & (N - 1), jp = (j + 1) & (N - 1);
            const double kp = Kp[k], km = Km[k];
            const double mm = 1.5 * double(n[jm]), m0 = 1.5 * double(n[j]), mp = 1.5 * double(n[jp]);
            const int pj = pad(j);
            A[pj] = -r * km / mm;
            B[pj] = 1.0 + r * (km + kp) / m0;
            Cc[pj] = -r * kp / mp;
            D[pj] = rhs_w[k];
        }
    }
    cyclic_reduce(A, B, Cc, D, N);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = threadIdx.x + k * kSolveBlock;
        if (j < N) w[j] = fmaxf(float(D[pad(j)]), 1.5f * n[j] * G.T_min);
    }
}

// the solve as a kernel of its own, after the face kernel (and, with the
// network flux closure, after the network): face values from memory
__global__ __launch_bounds__(kSolveBlock) void k_fluid_solve(Globals G)
{
    __shared__ double A[kPadCells], B[kPadCells], Cc[kPadCells], D[kPadCells];
    __shared__ float tab[kMaxTableRows * kCols];
    const ColDev C = G.cols[blockIdx.x];
    const int N = G.N;
    const int64_t o = int64_t(blockIdx.x) * N;
    const float* n = G.n + o;
    const float* w = G.w + o;
    const double dx = C.L / double(N);
    const double dt = double(G.dt);
    const double r = dt / (dx * dx);
    stage_table(G, tab);
    double rhs_w[kRows];
    float Kp[kRows], Km[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = threadIdx.x + k * kSolveBlock;
        rhs_w[k] = 0.0;
        Kp[k] = Km[k] = 0.0f;
        if (j < N) {
            const int jm = (j - 1) & (N - 1);
            float gp, gm, hp, hm;
            if (G.mlp == kNetFlux) {
                gp = G.y[(o + j) * 2] * G.norm[10] + G.norm[12];
                gm = G.y[(o + jm) * 2] * G.norm[10] + G.norm[12];
                hp = G.y[(o + j) * 2 + 1] * G.norm[11] + G.norm[13];
                hm = G.y[(o + jm) * 2 + 1] * G.norm[11] + G.norm[13];
            } else {
                gp = G.gam[o + j];
                gm = G.gam[o + jm];
                hp = G.H[o + j];
                hm = G.H[o + jm];
            }
            Kp[k] = G.kap[o + j];
            Km[k] = G.kap[o + jm];
            rhs_w[k] = setup_cell(G, C, tab, r, dt, dx, n[j], w[j], gp, gm, hp, hm, G.E[o + j], G.E[o + jm],
                                  G.Da[o + j], G.Da[o + jm], G.dn[o + j], G.dn[o + jm], Kp[k], Km[k], G.dT[o + j],
                                  G.dT[o + jm], pad(j), A, B, Cc, D);
        }
    }
    solve_tail(G, A, B, Cc, D, rhs_w, Kp, Km, r);
}

// faces and solve of one column in one workgroup (table and multiplier
// closures, whose fluxes the face pass computes): each cell's right face is
// the thread's own, its left face the neighbouring thread's, handed over
// through LDS that the tridiagonal systems take over afterwards.  The same
// arithmetic as the face kernel followed by the solve kernel, without the
// face arrays only the solve reads, their reload, a second table staging and
// a launch.
constexpr int kFaceVals = 7;
static_assert(kFaceVals * kMaxCells * sizeof(float) <= 4 * kPadCells * sizeof(double),
              "the face hand-over fits in the systems' LDS");
__global__ __launch_bounds__(kSolveBlock) void k_fluid_step(Globals G)
{
    __shared__ double sys[4 * kPadCells];
    __shared__ float tab[kMaxTableRows * kCols];
    __shared__ double sh[kFaceBlock / 64];
    double* A = sys;
    double* B = sys + kPadCells;
    double* Cc = sys + 2 * kPadCells;
    double* D = sys + 3 * kPadCells;
    float* X = reinterpret_cast<float*>(sys);   // [kFaceVals][N], before the systems are set up
    const ColDev C = G.cols[blockIdx.x];
    const int N = G.N;
    const int64_t o = int64_t(blockIdx.x) * N;
    const float* n = G.n + o;
    const float* w = G.w + o;
    const double dx = C.L / double(N);
    const double dt = double(G.dt);
    const double r = dt / (dx * dx);
    stage_table(G, tab);
    FaceOut fo[kFacesPerThread];
    faces_column(G, C, tab, sh, fo, false);
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = threadIdx.x + k * kSolveBlock;
        if (j < N) {
            X[0 * N + j] = fo[k].E;
            X[1 * N + j] = fo[k].Da;
            X[2 * N + j] = fo[k].kap;
            X[3 * N + j] = fo[k].dn;
            X[4 * N + j] = fo[k].dT;
            X[5 * N + j] = fo[k].gam;
            X[6 * N + j] = fo[k].H;
        }
    }
    __syncthreads();
    FaceOut fm[kRows];   // face j - 1 of each own cell j
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = threadIdx.x + k * kSolveBlock;
        if (j < N) {
            const int jm = (j - 1) & (N - 1);
            fm[k].E = X[0 * N + jm];
            fm[k].Da = X[1 * N + jm];
            fm[k].kap = X[2 * N + jm];
            fm[k].dn = X[3 * N + jm];
            fm[k].dT = X[4 * N + jm];
            fm[k].gam = X[5 * N + jm];
            fm[k].H = X[6 * N + jm];
        }
    }
    __syncthreads();   // the hand-over is read before the systems overwrite it
    double rhs_w[kRows];
    float Kp[kRows], Km[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = threadIdx.x + k * kSolveBlock;
        rhs_w[k] = 0.0;
        Kp[k] = Km[k] = 0.0f;
        if (j < N) {
            Kp[k] = fo[k].kap;
            Km[k] = fm[k].kap;
            rhs_w[k] = setup_cell(G, C, tab, r, dt, dx, n[j], w[j], fo[k].gam, fm[k].gam, fo[k].H, fm[k].H,
                                  fo[k].E, fm[k].E, fo[k].Da, fm[k].Da, fo[k].dn, fm[k].dn, Kp[k], Km[k], fo[k].dT,
                                  fm[k].dT, pad(j), A, B, Cc, D);
        }
    }
    solve_tail(G, A, B, Cc, D, rhs_w, Kp, Km, r);
}

// stand-alone batched cyclic tridiagonal solve (device arrays [ns][N]); x -> d
__global__ __launch_bounds__(kSolveBlock) void k_cyclic(const double* a, const double* b, const double* c,
                                                        double* d, int N)
{
    __shared__ double A[kPadCells], B[kPadCells], Cc[kPadCells], D[kPadCells];
    const int64_t o = int64_t(blockIdx.x) * N;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        A[pad(j)] = a[o + j];
        B[pad(j)] = b[o + j];
        Cc[pad(j)] = c[o + j];
        D[pad(j)] = d[o + j];
    }
    cyclic_reduce(A, B, Cc, D, N);
    for (int j = threadIdx.x; j < N; j += blockDim.x) d[o + j] = D[pad(j)];
}

}  // namespace pcfluid

// ---------------------------------------------------------------- C ABI
using namespace pcfluid;

struct pc_fluid {
    pc_fluid_config cfg;
    Globals G;
    hipStream_t st;
    const void* mlp_packed;
};

namespace {
thread_local const char* g_fluid_err = "";

pc_status ferr(pc_status s, const char* m)
{
    g_fluid_err = m;
    return s;
}

struct FLayout {
    int64_t cols, table, n, w, faces[7], x, y, total;
};

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

pc_status validate(const pc_fluid_config* c)
{
    if (!c) return ferr(PC_ERR_INVALID_ARG, "null config");
    if (c->n_columns < 1 || c->n_columns > 65535) return ferr(PC_ERR_INVALID_ARG, "n_columns");
    if (!pow2(c->n_cells) || c->n_cells < 64 || c->n_cells > kMaxCells)
        return ferr(PC_ERR_INVALID_ARG, "n_cells must be a power of two in [64, 4096]");
    if (c->table_len < 2 || c->table_len > kMaxTableRows)
        return ferr(PC_ERR_INVALID_ARG, "table_len must be in [2, 1024]");
    if (!(c->dt > 0.0) || !(c->T_step > 0.0) || !(c->T_min > 0.0) || !(c->n_floor > 0.0))
        return ferr(PC_ERR_INVALID_ARG, "dt, T_min, T_step and n_floor must be positive");
    return PC_OK;
}

FLayout flayout(const pc_fluid_config* c)
{
    FLayout L{};
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o = (o + bytes + 255) & ~int64_t(255);
        return at;
    };
    const int64_t cells = int64_t(c->n_columns) * c->n_cells;
    L.cols = take(int64_t(c->n_columns) * sizeof(ColDev));
    L.table = take(int64_t(c->table_len) * kCols * 4);
    L.n = take(cells * 4);
    L.w = take(cells * 4);
    for (int k = 0; k < 7; ++k) L.faces[k] = take(cells * 4);
    L.x = take(cells * 5 * 4);
    L.y = take(cells * 2 * 4);
    L.total = o;
    return L;
}
}  // namespace

extern "C" {

pc_status pc_fluid_query(const pc_fluid_config* cfg, int64_t* workspace_bytes)
{
    const pc_status s = validate(cfg);
    if (s != PC_OK) return s;
    if (!workspace_bytes) return ferr(PC_ERR_INVALID_ARG, "null output");
    *workspace_bytes = flayout(cfg).total;
    return PC_OK;
}

pc_status pc_fluid_init(const pc_fluid_config* cfg, const pc_fluid_column* cols, const double* table,
                        void* workspace, size_t bytes, void* hip_stream, pc_fluid_handle* out)
{
    pc_status s = validate(cfg);
    if (s != PC_OK) return s;
    if (!cols || !table || !workspace || !out) return ferr(PC_ERR_INVALID_ARG, "null argument");
    const FLayout L = flayout(cfg);
    if (int64_t(bytes) < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return ferr(PC_ERR_WORKSPACE, "workspace too small or misaligned");
    for (int c = 0; c < cfg->n_columns; ++c)
        if (!(cols[c].L > 0.0) || !(cols[c].Ngas > 0.0) || !(cols[c].muiN > 0.0) || !(cols[c].nu_w >= 0.0))
            return ferr(PC_ERR_INVALID_ARG, "column parameters");
    pc_fluid* h = new (std::nothrow) pc_fluid();
    if (!h) return ferr(PC_ERR_INVALID_ARG, "host allocation failed");
    h->cfg = *cfg;
    h->st = static_cast<hipStream_t>(hip_stream);
    char* b = static_cast<char*>(workspace);
    Globals& G = h->G;
    G.N = cfg->n_cells;
    G.K = cfg->table_len;
    G.mlp = kTable;
    G.have_m = 0;
    G.T_min = float(cfg->T_min);
    G.T_step = float(cfg->T_step);
    G.n_floor = float(cfg->n_floor);
    G.dt = float(cfg->dt);
    G.cols = reinterpret_cast<const ColDev*>(b + L.cols);
    G.table = reinterpret_cast<const float*>(b + L.table);
    G.n = reinterpret_cast<float*>(b + L.n);
    G.w = reinterpret_cast<float*>(b + L.w);
    float** fa[7] = {&G.gam, &G.H, &G.E, &G.Da, &G.kap, &G.dn, &G.dT};
    for (int k = 0; k < 7; ++k) *fa[k] = reinterpret_cast<float*>(b + L.faces[k]);
    G.x = reinterpret_cast<float*>(b + L.x);
    G.y = reinterpret_cast<const float*>(b + L.y);
    std::memset(G.norm, 0, sizeof(G.norm));
    std::vector<ColDev> cd(cfg->n_columns);
    for (int c = 0; c < cfg->n_columns; ++c)
        cd[c] = ColDev{cols[c].L, cols[c].Ngas, cols[c].E0, cols[c].nu_w, cols[c].muiN};
    std::vector<float> tf(size_t(cfg->table_len) * kCols);
    for (size_t k = 0; k < tf.size(); ++k) tf[k] = float(table[k]);
    hipError_t e = hipMemcpyAsync(b + L.cols, cd.data(), cd.size() * sizeof(ColDev), hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b + L.table, tf.data(), tf.size() * 4, hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) {
        delete h;
        return ferr(PC_ERR_HIP, "pc_fluid_init copies");
    }
    *out = h;
    return PC_OK;
}

pc_status pc_fluid_set_state(pc_fluid_handle h, const float* n, const float* w)
{
    if (!h || !n || !w) return ferr(PC_ERR_INVALID_ARG, "null argument");
    h->G.have_m = 0;   // multipliers answer the state's own past only
    const size_t bytes = size_t(h->cfg.n_columns) * h->cfg.n_cells * 4;
    if (hipMemcpyAsync(h->G.n, n, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess ||
        hipMemcpyAsync(h->G.w, w, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess)
        return ferr(PC_ERR_HIP, "pc_fluid_set_state");
    return PC_OK;
}

pc_status pc_fluid_get_state(pc_fluid_handle h, float* n, float* w)
{
    if (!h) return ferr(PC_ERR_INVALID_ARG, "null handle");
    const size_t bytes = size_t(h->cfg.n_columns) * h->cfg.n_cells * 4;
    if ((n && hipMemcpyAsync(n, h->G.n, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess) ||
        (w && hipMemcpyAsync(w, h->G.w, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess))
        return ferr(PC_ERR_HIP, "pc_fluid_get_state");
    return PC_OK;
}

pc_status pc_fluid_set_closure(pc_fluid_handle h, const void* mlp_packed, const float* norm)
{
    if (!h || (mlp_packed && !norm)) return ferr(PC_ERR_INVALID_ARG, "bad closure arguments");
    h->mlp_packed = mlp_packed;
    h->G.mlp = mlp_packed != nullptr ? kNetFlux : kTable;
    h->G.have_m = 0;
    if (norm) std::memcpy(h->G.norm, norm, sizeof(h->G.norm));
    return PC_OK;
}

pc_status pc_fluid_set_closure_multipliers(pc_fluid_handle h, const void* mlp_packed, const float* norm)
{
    if (!h || !mlp_packed || !norm) return ferr(PC_ERR_INVALID_ARG, "bad closure arguments");
    h->mlp_packed = mlp_packed;
    h->G.mlp = kNetMult;
    h->G.have_m = 0;
    std::memcpy(h->G.norm, norm, sizeof(h->G.norm));
    return PC_OK;
}

pc_status pc_fluid_step(pc_fluid_handle h, int64_t n_steps)
{
    if (!h || n_steps < 0) return ferr(PC_ERR_INVALID_ARG, "bad step arguments");
    const int nc = h->cfg.n_columns;
    const int64_t cells = int64_t(nc) * h->cfg.n_cells;
    for (int64_t k = 0; k < n_steps; ++k) {
        if (h->G.mlp == kNetFlux) {
            // the network gives this step's fluxes: faces, network, solve
            hipLaunchKernelGGL(k_fluid_faces, dim3(nc), dim3(kFaceBlock), 0, h->st, h->G);
            const pc_status s = pc_mlp_forward(h->mlp_packed, h->G.x, cells, const_cast<float*>(h->G.y), nullptr,
                                               h->st);
            if (s != PC_OK) return s;
            hipLaunchKernelGGL(k_fluid_solve, dim3(nc), dim3(kSolveBlock), 0, h->st, h->G);
        } else {
            // table fluxes (with the multipliers of the previous answer):
            // faces and solve in one kernel; the network then gives the
            // multipliers of the next step from this step's face inputs
            hipLaunchKernelGGL(k_fluid_step, dim3(nc), dim3(kSolveBlock), 0, h->st, h->G);
            if (h->G.mlp == kNetMult) {
                const pc_status s = pc_mlp_forward(h->mlp_packed, h->G.x, cells, const_cast<float*>(h->G.y),
                                                   nullptr, h->st);
                if (s != PC_OK) return s;
                h->G.have_m = 1;
            }
        }
    }
    return hipGetLastError() == hipSuccess ? PC_OK : ferr(PC_ERR_HIP, "pc_fluid_step launch");
}

pc_status pc_fluid_get_faces(pc_fluid_handle h, float* gamma, float* H, float* E)
{
    if (!h) return ferr(PC_ERR_INVALID_ARG, "null handle");
    const size_t bytes = size_t(h->cfg.n_columns) * h->cfg.n_cells * 4;
    if (h->G.mlp == kNetFlux && (gamma || H))
        return ferr(PC_ERR_INVALID_ARG, "network flux closure: fluxes are not stored");
    if ((gamma && hipMemcpyAsync(gamma, h->G.gam, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess) ||
        (H && hipMemcpyAsync(H, h->G.H, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess) ||
        (E && hipMemcpyAsync(E, h->G.E, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess))
        return ferr(PC_ERR_HIP, "pc_fluid_get_faces");
    return PC_OK;
}

pc_status pc_cyclic_tridiag(const double* a, const double* b, const double* c, double* d, int32_t n_systems,
                            int32_t n, void* hip_stream)
{
    if (!a || !b || !c || !d || n_systems < 1 || !pow2(n) || n < 2 || n > kMaxCells)
        return ferr(PC_ERR_INVALID_ARG, "bad tridiagonal arguments (n a power of two <= 4096)");
    hipLaunchKernelGGL(k_cyclic, dim3(n_systems), dim3(kSolveBlock), 0, static_cast<hipStream_t>(hip_stream), a, b,
                       c, d, n);
    return hipGetLastError() == hipSuccess ? PC_OK : ferr(PC_ERR_HIP, "pc_cyclic_tridiag launch");
}

void pc_fluid_destroy(pc_fluid_handle h) { delete h; }

const char* pc_fluid_last_error(void) { return g_fluid_err; }

}  // extern "C"
