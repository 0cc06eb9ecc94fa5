// kin_fluid.hip -- the fluid step of the operator-split reactive Euler solver (Sec. 3.1), on a
// 2-D grid whose cells hold the conserved variables of Sec. 2, Q = (rho_s [Ns], rho u, rho v, E),
// E = sum_s rho_s e_s + rho |u|^2 / 2 with each species' energy taken without its formation
// energy, e_s(T) = e_s^NASA(T) - e_s^NASA(T_ref), T_ref = 298.15 K (Sec. 2, Eq. energy); the
// chemistry sub-step of the split (the conserved-variable adapter) uses the same energy.
//
// A step is dimensionally split: an x sweep then a y sweep (or the reverse).  A sweep is three
// Runge-Kutta stages (the strong-stability-preserving third-order scheme), and a stage is three
// kernels, each bound by HBM bandwidth:
//   fluid_prim    per cell: Q -> primitive W = (rho_s, u, v, P) and T (Newton on the energy,
//                 from the cell's previous T), with P from Dalton's law (Sec. 2, Eq. dalton);
//   fluid_flux    per face: MP5 left and right states of every primitive variable (Sec. 3.1,
//                 Eq. mp5) with the monotonicity-preserving bound (Eqs. mp, ump), and the HLLE
//                 flux between them (Eq. fluxhlle);
//   fluid_update  per cell: the stage's combination of the sweep's start state, the stage state
//                 and dt times the flux difference.
// One thread per cell or face; consecutive threads take consecutive x, so every array access
// of a wavefront is one or two contiguous runs of a row.  The face kernel reads its six-cell
// stencil from the primitive array, which neighbouring threads share through the caches.
// Species are streamed (three passes per face), so no per-species array lives in registers.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kin_internal.h"
#include "kin_xlane.h"

namespace kin {
namespace {

constexpr double kRuJ = 8.31446261815324e3;   // J/(kmol K): R / M with M in g/mol gives J/(kg K)
constexpr double kAlphaMP = 2.0;
// Species counts whose face states and densities the kernels keep in registers, in two classes:
// the arrays are sized by the class, so a small mixture in the larger class would hold registers
// for species it does not have (the 9-species mixture's face kernel: 118 VGPRs and four
// wavefronts per SIMD in the small class, 142 and three in the larger).
constexpr int kFluidNsSmall = 10;
constexpr int kFluidNsRegs = 16;

__device__ __forceinline__ double minmod(double a, double b)
{
    return (a * b > 0.0) ? (a > 0.0 ? fmin(a, b) : fmax(a, b)) : 0.0;
}

// Left state of the face j + 1/2 from cells j-2..j+2 (Eq. mp5), limited by the median with u_j
// and u_j + minmod(u_{j+1} - u_j, alpha (u_j - u_{j-1})) (Eqs. mp, ump); the right state is the
// same function of the mirrored stencil.
__device__ __forceinline__ double mp5(double um2, double um1, double u0, double up1, double up2)
{
    const double uL = (2.0 * um2 - 13.0 * um1 + 47.0 * u0 + 27.0 * up1 - 3.0 * up2) / 60.0;
    const double ump = u0 + minmod(up1 - u0, kAlphaMP * (u0 - um1));
    return uL + minmod(u0 - uL, ump - uL);
}

// Sensible energy e_s(T) - e_s(T_ref) (J/kg) and c_v,s (J/(kg K)) of species s.  The species
// index is uniform across the wavefront, so both coefficient ranges come through scalar loads
// and each lane selects its range.
__device__ __forceinline__ void species_e_cv(const WaveTables &t, int s, double T, double &e, double &cv)
{
    const auto *nasa = uniform_table(t.nasa) + 14 * s;
    const bool lo = T < uniform_table(t.Tmid)[s];
    double a[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) a[k] = lo ? nasa[k] : nasa[7 + k];
    const double Rs = kRuJ / uniform_table(t.M)[s];
    const double cpR = fma(T, fma(T, fma(T, fma(T, a[4], a[3]), a[2]), a[1]), a[0]);
    const double hR = fma(T, fma(T, fma(T, fma(T, fma(T, a[4] * 0.2, a[3] * 0.25), a[2] * (1.0 / 3.0)), a[1] * 0.5), a[0]), a[5]);
    e = Rs * (hR - T) - uniform_table(t.ef)[s];
    cv = Rs * (cpR - 1.0);
}

struct Grid {
    int ns, nx, ny, bc;   // bc: 0 periodic, 1 zero-gradient
    long long n;          // nx * ny
};

// Primitive variables of cell i from its conserved state q (ns partial densities, two momenta,
// E; q(v) returns variable v): u, v, P = rho R T into W's last three rows and T into Tc, by
// Newton on the sensible energy from the cell's previous T.  The partial densities are W's
// species rows by definition, so the face kernel reads them from the state itself.
// NSR > 0: the partial densities stay in registers through the Newton iterations (mechanisms
// of at most NSR species); NSR = 0 reads them through q again in each iteration.
template <int NSR, typename QV>
__device__ __forceinline__ void cell_primitives(const WaveTables &t, const Grid &g, long long i, QV q, double *W,
                                                double *Tc)
{
    const int ns = g.ns;
    const long long n = g.n;
    double rs[NSR > 0 ? NSR : 1];
    auto each_species = [&](auto body) {
        if constexpr (NSR > 0) {
#pragma unroll
            for (int s = 0; s < NSR; ++s)
                if (s < ns) body(s);
        } else {
            for (int s = 0; s < ns; ++s) body(s);
        }
    };
    auto rho_s = [&](int s) { return NSR > 0 ? rs[s] : q(s); };
    double rho = 0.0, rR = 0.0;
    each_species([&](int s) {
        const double r = q(s);
        if constexpr (NSR > 0) rs[s] = r;
        rho += r;
        rR = fma(r, kRuJ / uniform_table(t.M)[s], rR);
    });
    const double u = q(ns) / rho, v = q(ns + 1) / rho;
    const double eint = q(ns + 2) - 0.5 * rho * (u * u + v * v);
    double T = Tc[i];
    if (!(T >= 100.0 && T <= 1e4)) T = 1000.0;
    if constexpr (NSR > 0) {
        // Within one choice of NASA-7 range per species the mixture's sensible energy is itself
        // a polynomial in T: with w_s = rho_s R_s and B_k = sum_s w_s a_sk, sum_s rho_s e_s(T) =
        // B_5 + T (B_0 + T (B_1 / 2 + ... + T B_4 / 5)) - rR T - sum_s rho_s ef_s, and the heat
        // capacity is B_0 + T (B_1 + ... + T B_4) - rR.  The B_k are summed once per range choice
        // (a bit per species, set below its switch temperature), so a Newton iteration costs one
        // polynomial instead of one per species.
        static_assert(NSR <= 32, "range mask");
        double B[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, EF = 0.0;
        each_species([&](int s) { EF = fma(rs[s], uniform_table(t.ef)[s], EF); });
        unsigned used = ~0u;  // no valid choice yet (ns <= 16 < 32 bits)
        for (int it = 0; it < 60; ++it) {
            unsigned lo = 0;
            each_species([&](int s) { lo |= (T < uniform_table(t.Tmid)[s] ? 1u : 0u) << s; });
            if (lo != used) {
                used = lo;
#pragma unroll
                for (int k = 0; k < 6; ++k) B[k] = 0.0;
                each_species([&](int s) {
                    const auto *nasa = uniform_table(t.nasa) + 14 * s;
                    const bool l = (lo >> s) & 1u;
                    const double w = rs[s] * (kRuJ / uniform_table(t.M)[s]);
#pragma unroll
                    for (int k = 0; k < 6; ++k) B[k] = fma(w, l ? nasa[k] : nasa[7 + k], B[k]);
                });
            }
            const double C = fma(T, fma(T, fma(T, fma(T, B[4], B[3]), B[2]), B[1]), B[0]);
            const double H = fma(T, fma(T, fma(T, fma(T, fma(T, B[4] * 0.2, B[3] * 0.25), B[2] * (1.0 / 3.0)),
                                                B[1] * 0.5), B[0]), B[5]);
            const double f = H - rR * T - EF - eint;
            const double d = C - rR;
            const double dT = f / d;
            T -= dT;
            if (!(fabs(dT) > 1e-13 * fabs(T))) break;   // converged, or not a number
        }
    } else {
        for (int it = 0; it < 60; ++it) {
            double f = -eint, d = 0.0;
            each_species([&](int s) {
                double e, cv;
                species_e_cv(t, s, T, e, cv);
                const double r = rho_s(s);
                f = fma(r, e, f);
                d = fma(r, cv, d);
            });
            const double dT = f / d;
            T -= dT;
            if (!(fabs(dT) > 1e-13 * fabs(T))) break;   // converged, or not a number
        }
    }
    Tc[i] = T;
    W[(size_t)ns * n + i] = u;
    W[(size_t)(ns + 1) * n + i] = v;
    W[(size_t)(ns + 2) * n + i] = rR * T;
}

template <int NSR>
__global__ void fluid_prim_kernel(WaveTables t, Grid g, const double *Q, double *W, double *Tc)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const long long n = g.n;
    cell_primitives<NSR>(t, g, i, [&](int v) { return Q[(size_t)v * n + i]; }, W, Tc);
}

// Cell index along the sweep direction k (0..len-1 after the boundary rule) of an offset one.
__device__ __forceinline__ int wrap(int k, int len, int bc)
{
    if (bc == 0) return k < 0 ? k + len : (k >= len ? k - len : k);
    return k < 0 ? 0 : (k >= len ? len - 1 : k);
}

// Face fluxes of a sweep along x (DIR 0) or y (DIR 1).  Face a along the sweep lies between
// cells a - 1 and a; faces are stored [var][ny][nx + 1] (x) or [var][ny + 1][nx] (y).
// NSR > 0: mechanisms of at most NSR species keep each species' two reconstructed states in
// registers (one reconstruction per species); NSR = 0 streams them (three per species).
template <int DIR, int NSR>
__global__ void __launch_bounds__(256) fluid_flux_kernel(WaveTables t, Grid g, const double *Qs, const double *W, double *F)
{
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int fw = DIR == 0 ? g.nx + 1 : g.nx;      // faces per row of the face array
    const int fh = DIR == 0 ? g.ny : g.ny + 1;
    if (f >= (long long)fw * fh) return;
    const int fx = (int)(f % fw), fy = (int)(f / fw);
    const int a = DIR == 0 ? fx : fy;                 // face index along the sweep
    const int len = DIR == 0 ? g.nx : g.ny;
    const long long n = g.n;
    const int ns = g.ns;
    // cells a-3 .. a+2 along the sweep (j = a - 1 is the face's left cell)
    long long c[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int q = wrap(a - 3 + k, len, g.bc);
        c[k] = DIR == 0 ? (long long)fy * g.nx + q : (long long)q * g.nx + fx;
    }
    auto recon = [&](const double *w, double &L, double &R) {
        const double v0 = w[c[0]], v1 = w[c[1]], v2 = w[c[2]], v3 = w[c[3]], v4 = w[c[4]], v5 = w[c[5]];
        L = mp5(v0, v1, v2, v3, v4);
        R = mp5(v5, v4, v3, v2, v1);
    };
    const double *Wun = W + (size_t)(DIR == 0 ? ns : ns + 1) * n;
    const double *Wut = W + (size_t)(DIR == 0 ? ns + 1 : ns) * n;
    double unL, unR, utL, utR, PL, PR;
    recon(Wun, unL, unR);
    recon(Wut, utL, utR);
    recon(W + (size_t)(ns + 2) * n, PL, PR);
    // species states: reconstructed once into registers (NSR), or again in each pass below
    double Ls[NSR > 0 ? NSR : 1], Rsv[NSR > 0 ? NSR : 1];
    if (NSR > 0) {
#pragma unroll
        for (int s = 0; s < (NSR > 0 ? NSR : 1); ++s)
            if (s < ns) recon(Qs + (size_t)s * n, Ls[s], Rsv[s]);
    }
    auto state = [&](int s, double &L, double &R) {
        if (NSR > 0) {
            L = Ls[s];
            R = Rsv[s];
        } else {
            recon(Qs + (size_t)s * n, L, R);
        }
    };
    // body(s) for every species: unrolled over the register arrays, or a plain loop
    auto each_species = [&](auto body) {
        if constexpr (NSR > 0) {
#pragma unroll
            for (int s = 0; s < NSR; ++s)
                if (s < ns) body(s);
        } else {
            for (int s = 0; s < ns; ++s) body(s);
        }
    };
    // pass 1: densities and gas constants of the two states
    double rL = 0.0, rR = 0.0, RL = 0.0, RR = 0.0;
    each_species([&](int s) {
        double L, R;
        state(s, L, R);
        const double Rs = kRuJ / uniform_table(t.M)[s];
        rL += L;
        rR += R;
        RL = fma(L, Rs, RL);
        RR = fma(R, Rs, RR);
    });
    const double TL = PL / RL, TR = PR / RR;
    // pass 2: energies and heat capacities at the two temperatures
    double eL = 0.0, eR = 0.0, cvL = 0.0, cvR = 0.0;
    each_species([&](int s) {
        double L, R, e, cv;
        state(s, L, R);
        species_e_cv(t, s, TL, e, cv);
        eL = fma(L, e, eL);
        cvL = fma(L, cv, cvL);
        species_e_cv(t, s, TR, e, cv);
        eR = fma(R, e, eR);
        cvR = fma(R, cv, cvR);
    });
    const double EL = eL + 0.5 * rL * (unL * unL + utL * utL);
    const double ER = eR + 0.5 * rR * (unR * unR + utR * utR);
    const double cL = sqrt((cvL + RL) / cvL * PL / rL), cR = sqrt((cvR + RR) / cvR * PR / rR);
    const double sL = sqrt(rL), sR = sqrt(rR);
    const double uh = (sL * unL + sR * unR) / (sL + sR);
    const double c2h = (sL * cL * cL + sR * cR * cR) / (sL + sR) +
                       0.5 * sL * sR / ((sL + sR) * (sL + sR)) * (unR - unL) * (unR - unL);
    const double ch = sqrt(c2h);
    const double bp = fmax(0.0, fmax(uh + ch, unR + cR));
    const double bm = fmin(0.0, fmin(uh - ch, unL - cL));
    const double idb = 1.0 / (bp - bm), pm = bp * bm * idb;
    auto hlle = [&](double FL, double FR, double QL, double QR) { return (bp * FL - bm * FR) * idb + pm * (QR - QL); };
    const long long fo = DIR == 0 ? (long long)fy * (g.nx + 1) + fx : (long long)fy * g.nx + fx;
    const long long fn = (long long)fw * fh;
    // pass 3: species fluxes
    each_species([&](int s) {
        double L, R;
        state(s, L, R);
        F[(size_t)s * fn + fo] = hlle(L * unL, R * unR, L, R);
    });
    F[(size_t)(DIR == 0 ? ns : ns + 1) * fn + fo] =
        hlle(rL * unL * unL + PL, rR * unR * unR + PR, rL * unL, rR * unR);
    F[(size_t)(DIR == 0 ? ns + 1 : ns) * fn + fo] = hlle(rL * unL * utL, rR * unR * utR, rL * utL, rR * utR);
    F[(size_t)(ns + 2) * fn + fo] = hlle(unL * (EL + PL), unR * (ER + PR), EL, ER);
}

// Qout = a0 Q0 + a1 (Q + dt L), L = -(F_{a+1} - F_a) / h (in place allowed: each thread reads
// and writes only its own cell).
template <int DIR>
__global__ void fluid_update_kernel(Grid g, const double *Q0, const double *Q, double *Qout, const double *F,
                                    double dt, double h, double a0, double a1)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const int x = (int)(i % g.nx), y = (int)(i / g.nx);
    const int nv = g.ns + 3;
    const long long fn = DIR == 0 ? (long long)(g.nx + 1) * g.ny : (long long)g.nx * (g.ny + 1);
    const long long fl = DIR == 0 ? (long long)y * (g.nx + 1) + x : i;
    const long long fr = DIR == 0 ? fl + 1 : fl + g.nx;
    for (int v = 0; v < nv; ++v) {
        const double L = -(F[(size_t)v * fn + fr] - F[(size_t)v * fn + fl]) / h;
        const double q = Q[(size_t)v * g.n + i] + dt * L;
        Qout[(size_t)v * g.n + i] = a0 != 0.0 ? a0 * Q0[(size_t)v * g.n + i] + a1 * q : a1 * q;
    }
}

// The update of fluid_update_kernel, then the primitives of the new state for the next stage
// (the new state stays in registers, so it is not read back).
template <int DIR, int NSR>
__global__ void fluid_update_prim_kernel(WaveTables t, Grid g, const double *Q0, const double *Q, double *Qout,
                                         const double *F, double dt, double h, double a0, double a1, double *W,
                                         double *Tc)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const int x = (int)(i % g.nx), y = (int)(i / g.nx);
    const int nv = g.ns + 3;
    const long long fn = DIR == 0 ? (long long)(g.nx + 1) * g.ny : (long long)g.nx * (g.ny + 1);
    const long long fl = DIR == 0 ? (long long)y * (g.nx + 1) + x : i;
    const long long fr = DIR == 0 ? fl + 1 : fl + g.nx;
    constexpr int NV = NSR > 0 ? NSR + 3 : 1;
    double qn[NV];
    auto upd = [&](int v) {
        const double L = -(F[(size_t)v * fn + fr] - F[(size_t)v * fn + fl]) / h;
        const double q = Q[(size_t)v * g.n + i] + dt * L;
        const double o = a0 != 0.0 ? a0 * Q0[(size_t)v * g.n + i] + a1 * q : a1 * q;
        Qout[(size_t)v * g.n + i] = o;
        return o;
    };
    if constexpr (NSR > 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            // species k < ns, then the momenta and the energy in slots NSR .. NSR + 2
            const int v = k < NSR ? k : g.ns + (k - NSR);
            if (k < NSR && k >= g.ns) continue;
            qn[k] = upd(v);
        }
        cell_primitives<NSR>(t, g, i, [&](int v) { return v < g.ns ? qn[v] : qn[NSR + (v - g.ns)]; }, W, Tc);
    } else {
        for (int v = 0; v < nv; ++v) upd(v);
        const long long n = g.n;
        cell_primitives<0>(t, g, i, [&](int v) { return Qout[(size_t)v * n + i]; }, W, Tc);
    }
}

// Largest (|u| + c) / dx and (|v| + c) / dy over the grid (positive doubles order like their
// bit patterns, so an unsigned 64-bit atomic maximum finds it).  A block strides over the grid
// and reduces its cells first, so the one word takes one atomic per block, not per wavefront.
constexpr int kSpeedThreads = 256;
constexpr int kSpeedBlocks = 1024;

__global__ void __launch_bounds__(kSpeedThreads) fluid_speed_kernel(WaveTables t, Grid g, const double *Q,
                                                                    const double *W, const double *Tc, double dx,
                                                                    double dy, unsigned long long *out)
{
    __shared__ double wmax[kSpeedThreads / 64];
    double r = 0.0;
    for (long long i = (long long)blockIdx.x * kSpeedThreads + threadIdx.x; i < g.n;
         i += (long long)gridDim.x * kSpeedThreads) {
        const long long n = g.n;
        double rho = 0.0, rR = 0.0, cv = 0.0;
        const double T = Tc[i];
        for (int s = 0; s < g.ns; ++s) {
            const double rs = Q[(size_t)s * n + i];
            double e, cvs;
            species_e_cv(t, s, T, e, cvs);
            rho += rs;
            rR = fma(rs, kRuJ / t.M[s], rR);
            cv = fma(rs, cvs, cv);
        }
        const double P = W[(size_t)(g.ns + 2) * n + i];
        const double c = sqrt((cv + rR) / cv * P / rho);
        double ri = fmax((fabs(W[(size_t)g.ns * n + i]) + c) / dx, (fabs(W[(size_t)(g.ns + 1) * n + i]) + c) / dy);
        if (!(ri >= 0.0)) ri = __builtin_inf();   // a bad cell makes the step size zero
        r = fmax(r, ri);
    }
    for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kSpeedThreads / 64; ++w) r = fmax(r, wmax[w]);
        atomicMax(out, (unsigned long long)__double_as_longlong(r));
    }
}

// Kinetic energy of each cell (kept for the way back), and E - KE, the energy the chemistry
// sub-step sees; after it, E = E_sens + KE with the same KE (chemistry changes neither the
// density nor the momentum).
__global__ void fluid_kinetic_kernel(Grid g, const double *Q, double *KE, double *Es)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const long long n = g.n;
    double rho = 0.0;
    for (int s = 0; s < g.ns; ++s) rho += Q[(size_t)s * n + i];
    const double mx = Q[(size_t)g.ns * n + i], my = Q[(size_t)(g.ns + 1) * n + i];
    const double ke = 0.5 * (mx * mx + my * my) / rho;
    KE[i] = ke;
    Es[i] = Q[(size_t)(g.ns + 2) * n + i] - ke;
}

__global__ void fluid_energy_back_kernel(Grid g, double *Q, const double *KE, const double *Es)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    Q[(size_t)(g.ns + 2) * g.n + i] = Es[i] + KE[i];
}

// f(std::integral_constant<int, NSR>) with the register class of ns species (0: streamed).
template <typename Fn>
void ns_class(int ns, Fn f)
{
    if (ns <= kFluidNsSmall) f(std::integral_constant<int, kFluidNsSmall>{});
    else if (ns <= kFluidNsRegs) f(std::integral_constant<int, kFluidNsRegs>{});
    else f(std::integral_constant<int, 0>{});
}

}  // namespace

hipError_t launch_fluid_sweep(const WaveTables &t, const FluidGrid &fg, int dir, double dt, double h,
                              double *Q, double *Q1, double *W, double *T, double *F, hipStream_t s)
{
    const Grid g{t.ns, fg.nx, fg.ny, fg.bc, (long long)fg.nx * fg.ny};
    const int block = 256;
    const unsigned gc = (unsigned)((g.n + block - 1) / block);
    const long long nf = dir == 0 ? (long long)(g.nx + 1) * g.ny : (long long)g.nx * (g.ny + 1);
    const unsigned gf = (unsigned)((nf + block - 1) / block);
    // (a0, a1, stage input, stage output): Q1 = Q + dt L(Q); Q1 <- 3/4 Q + 1/4 (Q1 + dt L(Q1));
    // Q <- 1/3 Q + 2/3 (Q1 + dt L(Q1))
    const double a0[3] = {0.0, 0.75, 1.0 / 3.0}, a1[3] = {1.0, 0.25, 2.0 / 3.0};
    // stage k: faces of its input's primitives, then the update, which in stages 0 and 1 also
    // forms the primitives of its output for the next stage
    ns_class(g.ns, [&](auto nsrc) {
        constexpr int NSR = decltype(nsrc)::value;
        hipLaunchKernelGGL((fluid_prim_kernel<NSR>), dim3(gc), dim3(block), 0, s, t, g, Q, W, T);
        auto stage = [&](auto dirc, const double *in, double *out, int k) {
            constexpr int D = decltype(dirc)::value;
            hipLaunchKernelGGL((fluid_flux_kernel<D, NSR>), dim3(gf), dim3(block), 0, s, t, g, in, W, F);
            if (k == 2)
                hipLaunchKernelGGL(fluid_update_kernel<D>, dim3(gc), dim3(block), 0, s, g, Q, in, out, F, dt, h, a0[k],
                                   a1[k]);
            else
                hipLaunchKernelGGL((fluid_update_prim_kernel<D, NSR>), dim3(gc), dim3(block), 0, s, t, g, Q, in, out, F,
                                   dt, h, a0[k], a1[k], W, T);
        };
        for (int k = 0; k < 3; ++k) {
            const double *in = k == 0 ? Q : Q1;
            double *out = k == 2 ? Q : Q1;
            if (dir == 0) stage(std::integral_constant<int, 0>{}, in, out, k);
            else stage(std::integral_constant<int, 1>{}, in, out, k);
        }
    });
    return hipGetLastError();
}

hipError_t launch_fluid_speed(const WaveTables &t, const FluidGrid &fg, const double *Q, double *W, double *T,
                              double dx, double dy, unsigned long long *out, hipStream_t s)
{
    const Grid g{t.ns, fg.nx, fg.ny, fg.bc, (long long)fg.nx * fg.ny};
    const int block = 256;
    const unsigned gc = (unsigned)((g.n + block - 1) / block);
    ns_class(g.ns, [&](auto nsrc) {
        constexpr int NSR = decltype(nsrc)::value;
        hipLaunchKernelGGL((fluid_prim_kernel<NSR>), dim3(gc), dim3(block), 0, s, t, g, Q, W, T);
    });
    const long long sb = (g.n + kSpeedThreads - 1) / kSpeedThreads;
    hipLaunchKernelGGL(fluid_speed_kernel, dim3((unsigned)(sb < kSpeedBlocks ? sb : kSpeedBlocks)), dim3(kSpeedThreads),
                       0, s, t, g, Q, W, T, dx, dy, out);
    return hipGetLastError();
}

hipError_t launch_fluid_kinetic(const FluidGrid &fg, int ns, const double *Q, double *KE, double *Es, hipStream_t s)
{
    const Grid g{ns, fg.nx, fg.ny, fg.bc, (long long)fg.nx * fg.ny};
    const int block = 256;
    hipLaunchKernelGGL(fluid_kinetic_kernel, dim3((unsigned)((g.n + block - 1) / block)), dim3(block), 0, s, g, Q, KE, Es);
    return hipGetLastError();
}

hipError_t launch_fluid_energy_back(const FluidGrid &fg, int ns, double *Q, const double *KE, const double *Es,
                                    hipStream_t s)
{
    const Grid g{ns, fg.nx, fg.ny, fg.bc, (long long)fg.nx * fg.ny};
    const int block = 256;
    hipLaunchKernelGGL(fluid_energy_back_kernel, dim3((unsigned)((g.n + block - 1) / block)), dim3(block), 0, s, g, Q, KE, Es);
    return hipGetLastError();
}

}  // namespace kin
