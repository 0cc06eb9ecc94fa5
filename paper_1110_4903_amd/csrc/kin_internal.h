// kin_internal.h -- host-side structures shared by the libkin translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "kin.h"

namespace kin {

constexpr int kNsMax = 255;         // species of a mechanism (the global-memory layout)
constexpr int kWaveNsMax = 63;      // N = Ns + 1 <= 64: one matrix row per wavefront lane
constexpr int kLaneNsMax = 15;      // lane layout holds the whole matrix in registers
// LDS of a lane-layout block: per wavefront a queue of 64 cells ((Ns + 4) doubles and 4
// integers each) and the 64 lanes' sub-step start states (Ns + 1 doubles each)
inline size_t lane_lds_bytes(int ns, int block) { return (size_t)(block / 64) * 64 * 8 * (2 * (ns + 1) + 7); }
inline bool lane_block_ok(int ns, int block)
{
    return ns <= kLaneNsMax && (block == 64 || block == 128 || block == 256) && lane_lds_bytes(ns, block) <= 65536;
}
constexpr double kRu = 8.31446261815324;          // J/(mol K)
constexpr double kRuCgs = 8.31446261815324e7;     // erg/(mol K)
constexpr double kPatmCgs = 1.01325e6;            // dyn/cm^2 (one standard atmosphere)

// One species taking part in a reaction, with its reactant, product and net coefficients.
struct Part {
    int sp;
    int nu_r;   // nu'  (reactant side)
    int nu_p;   // nu'' (product side)
    int nu;     // nu'' - nu'
};

struct Rxn {
    double A, lnA, b, Ta;
    int rev;     // 1: reverse rate through the equilibrium constant
    int tb;      // -1 or row of the efficiency table
    int dnu;     // sum nu'' - sum nu' over species
    int nreac, nprod, npart;
    int reac_sp[3], reac_nu[3];  // merged by species
    int prod_sp[3], prod_nu[3];
    Part part[6];
};

// Validated, preprocessed copy of a kin_mech_desc.
struct MechHost {
    int ns = 0, ne = 0, nr = 0, ntb = 0;
    std::vector<double> M, nasa, Tmid;
    std::vector<int8_t> elem;
    std::vector<Rxn> rx;
    std::vector<double> eff;
    bool single_range(int s) const;  // both NASA sets identical
};

// Validate d and build the preprocessed copy.  Returns KIN_OK or KIN_EINVAL with msg set.
kin_status mech_from_desc(const kin_mech_desc *d, MechHost &m, std::string &msg);

// Source of the lane-layout module for a mechanism: generated mechanism functions followed
// by the hand-written template.  block = threads per block.  consts receives the table of
// FP64 constants the generated code reads as K[i].
std::string lane_source(const MechHost &m, int block, std::vector<double> &consts);

// Compile HIP source for gfx950 with hipRTC.  Returns KIN_OK and the code object, or
// KIN_ECOMPILE with the log in msg.
kin_status rtc_compile(const std::string &src, const char *name, std::vector<char> &code,
                       std::string &msg, double *seconds);

void set_error(const std::string &msg);

}  // namespace kin

namespace kin {

// Mechanism tables in device memory, read by the table-driven kernels (wave layout and the
// initial-energy kernel).  All pointers point into one allocation.
constexpr int kChunk = 64;   // reactions evaluated per wavefront pass

// Compact reaction record (48 bytes).  A reaction has six species slots: reactants in slots
// 0-2 and products in slots 3-5 (species merged within each side; unused slots have nu = 0
// and species 0).  nu holds the slot's signed stoichiometric coefficient (-nu' for a reactant,
// +nu'' for a product); coff and roff are byte offsets of the slot's species in a species
// vector (8 s) and of its row in the Jacobian (8 s (NPAD + 1), NPAD the padded row length).
struct RxnRec {
    int8_t rev, pad0;
    int16_t tb;
    int8_t nu[6];
    int8_t pad1[2];
    uint16_t coff[6];
    uint16_t roff[6];
    int8_t pad2[12];
};
static_assert(sizeof(RxnRec) == 48, "reaction record must stay 48 bytes");

// Per-reaction coefficients of the Jacobian scatter, one entry per slot: the row factor
// nu M_s (signed, zero for unused slots) and the column factor 1 / M_s (zero for unused slots).
struct RxnCoef {
    double rowc[6];
    double colc[6];
};

struct WaveTables {
    int ns, nr, ntb, nchunk;  // ntb: third-body reactions (each has a slot; RxnRec::tb is the slot)
    int ntbe;                 // third-body Jacobian entries (slot, row) over all slots
    int tb_last;              // slots 0..tb_last-1 have a participant in the wave layout's last
                              // 16-row tile (the slots are numbered so)
    double lnPaR;           // ln(P_atm / R) in CGS units
    const double *nasa;     // [ns][14]
    const double *Tmid;     // [ns]
    const double *M;        // [ns] g/mol
    // reaction tables are stored in order of (reactant count, product count), not in the
    // mechanism's order
    const double *rxd;      // [nr][4]: ln A, b, Ta, sum nu
    const RxnRec *rxc;      // [nr]
    const RxnCoef *rxk;     // [nr]
    const double *ef;       // [ns] e_s(T_ref) at T_ref = 298.15 K, J/kg (conserved-variable adapter)
    const double *effT;     // [ns][ntb] third-body efficiencies per slot, transposed
    const double *tbA;      // [ceil(ntb/4)][ceil(ns/16)][64] nu_qs M_s in matrix-operand tiles
    const double *tbB;      // [ceil(ntb/4)][ceil(ns/16)][64] eff_qk / M_k in matrix-operand tiles
    const int *tgs;         // [ntbe] the same entries ordered by slot: slot | row << 16
    const double *tgf;      // [ntbe] row factor nu_rs M_s of each tgs entry
    const double *effTM;    // [ns][ntb] effT[k][q] / M_k
    const int *chunk_rp;    // [nchunk] largest reactant count | largest product count << 8, per
                            // pass of 64 reactions
};

// Device layout of one instance's arena (n cells, ns species), from its base address:
//   rho[n] e0[n] T[n] Y[ns][n] sched[n] (8-byte entries, each array 256-byte aligned)
//   status[n] level[n] iters[n] (4-byte entries), one 64-bit work counter, the cell order
//   order[n] of a cost-ordered advance, its per-tile class counts ocount[8 * tiles] and the
//   cost classes okey[n] of a first advance (no iteration counts yet).
struct Arena {
    double *rho, *e0, *T, *Y;
    unsigned long long *sched;
    int *status, *level, *iters;
    unsigned long long *counter;
    int *order, *ocount, *okey;
};

// Cost-ordered advance: cells are classed by their Newton iterations in the previous advance
// (kOrderClasses classes) in tiles of kOrderTile cells.
constexpr int kOrderTile = 2048;
constexpr int kOrderClasses = 8;
__host__ __device__ inline long long order_tiles(long long n) { return (n + kOrderTile - 1) / kOrderTile; }

__host__ __device__ inline size_t arena_align(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline Arena arena_at(char *base, long long n, int ns)
{
    const size_t d = arena_align(sizeof(double) * (size_t)n);
    const size_t i = arena_align(sizeof(int) * (size_t)n);
    Arena a;
    a.rho = reinterpret_cast<double *>(base);
    a.e0 = reinterpret_cast<double *>(base + d);
    a.T = reinterpret_cast<double *>(base + 2 * d);
    a.Y = reinterpret_cast<double *>(base + 3 * d);
    a.sched = reinterpret_cast<unsigned long long *>(base + (3 + (size_t)ns) * d);
    char *ib = base + (4 + (size_t)ns) * d;
    a.status = reinterpret_cast<int *>(ib);
    a.level = reinterpret_cast<int *>(ib + i);
    a.iters = reinterpret_cast<int *>(ib + 2 * i);
    a.counter = reinterpret_cast<unsigned long long *>(ib + 3 * i);
    a.order = reinterpret_cast<int *>(ib + 3 * i + 256);
    a.ocount = reinterpret_cast<int *>(ib + 4 * i + 256);
    a.okey = reinterpret_cast<int *>(ib + 4 * i + 256 + arena_align(sizeof(int) * kOrderClasses * (size_t)order_tiles(n)));
    return a;
}

__host__ __device__ inline size_t arena_bytes(long long n, int ns)
{
    return arena_align(sizeof(double) * (size_t)n) * (4 + (size_t)ns) +
           5 * arena_align(sizeof(int) * (size_t)n) + 256 +
           arena_align(sizeof(int) * kOrderClasses * (size_t)order_tiles(n));
}

// One instance's share of an advance launch: cells [start, start + n) of the launch's global
// cell index space live in the arena at base, advanced by dt.
struct CellSpan {
    long long start, n;
    double dt;
    char *base;
    const int *order;  // position -> cell of the instance (cost order), or null: index order
};
constexpr int kMaxSpans = 64;

// Arguments of one advance launch (both layouts), passed by value; mirrors the device-side
// argument struct of the generated lane-layout module.
struct AdvanceArgs {
    CellSpan span[kMaxSpans];
    int nspan, ns;
    long long total;                 // cells over all spans
    double rtol, atol_Y, atol_T, y_neg;
    int k_max, L_max, L_forced, max_iters;
    int point_implicit;              // 1: accept the first (linearised) update as it is
    double diverge_ratio;            // > 0: fail an attempt whose update norm grows by more
    const double *K;                 // lane layout: the mechanism's constant table
    unsigned long long *counter;     // next unclaimed cell (zero at launch)
    // diagnostic sub-step schedule of every cell, or null: trace[g * trace_words + w] for the
    // cell at launch position g (span start + cell): word 0 the number of sub-step attempts,
    // words 1.. their accept bits (attempt j: bit j % 64 of word 1 + j / 64), recorded up to
    // 64 (trace_words - 1) attempts
    unsigned long long *trace;
    int trace_words;
};

// Fixed device memory of the allocation-free advance (kin_global.hip): kScratchLaunches 64-bit
// work counters at offset 0, then the global layout's matrix workspace from offset
// kScratchWorkOffset to the end.  256 MiB per device.
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kScratchLaunches = 64;
constexpr size_t kScratchWorkOffset = 4096;
constexpr int kScratchMaxDevices = 64;
// Device address of the fixed memory on `device`, which must be current.  Looked up once per
// device and kept.
hipError_t scratch_address(int device, unsigned char **out);

// Fluid grid (kin_fluid.hip): nx x ny cells, conserved variables [ns + 3][ny][nx]; bc 0 periodic,
// 1 zero-gradient (transmissive) in both directions.
struct FluidGrid {
    int nx, ny, bc;
};
// One dimensionally split sweep (dir 0 = x, 1 = y) of dt: three Runge-Kutta stages of the MP5 /
// HLLE update, Q in place; Q1 (stage state), W (primitives), T (temperatures, also the Newton
// start values) and F (face fluxes, (ns + 3) (nx + 1) (ny + 1) doubles) are workspace.
hipError_t launch_fluid_sweep(const WaveTables &t, const FluidGrid &g, int dir, double dt, double h, double *Q,
                              double *Q1, double *W, double *T, double *F, hipStream_t s);
// Largest (|u| + c) / dx, (|v| + c) / dy over the grid into *out (bit pattern, zero beforehand).
hipError_t launch_fluid_speed(const WaveTables &t, const FluidGrid &g, const double *Q, double *W, double *T,
                              double dx, double dy, unsigned long long *out, hipStream_t s);
// KE = rho |u|^2 / 2 and Es = E - KE per cell; and back, E = Es + KE.
hipError_t launch_fluid_kinetic(const FluidGrid &g, int ns, const double *Q, double *KE, double *Es, hipStream_t s);
hipError_t launch_fluid_energy_back(const FluidGrid &g, int ns, double *Q, const double *KE, const double *Es,
                                    hipStream_t s);

// Host launchers of the precompiled kernels (kin_wave.hip).
int wave_npad(int n);
hipError_t launch_conserved_in(const WaveTables &t, long long n, long long ld, double *rho, double *T,
                               double *Y, double *e0, bool have_guess, hipStream_t s);
hipError_t launch_conserved_out(const WaveTables &t, long long n, long long ld, const double *rho,
                                const double *Y, const double *e0, double *rho_s, double *E_sens,
                                hipStream_t s);
// Global-memory layout (kin_global.hip): workspace doubles per slot, and the launch over
// `slots` threads with a workspace of slots * global_work_doubles_per_slot doubles.
size_t global_work_doubles_per_slot(int ns, int ntb);
// Cost order of an instance's n cells (kin_order.hip): order[n], per-tile scratch
// ocount[kOrderClasses * order_tiles(n)].  key: the iterations of the previous advance, or
// with direct, cost classes 0..kOrderClasses-1 already.
// clear (may be null): a work counter that the order's scan sets to zero on the way
hipError_t launch_cost_order(const int *key, long long n, bool direct, int *order, int *ocount,
                              unsigned long long *clear, hipStream_t s);
hipError_t launch_global(const WaveTables &t, const AdvanceArgs &a, bool fp32_lu, double *work,
                         long long slots, hipStream_t stream);
hipError_t launch_energy(const WaveTables &t, long long n, long long ld, const double *T,
                         const double *Y, double *e0, hipStream_t stream);
hipError_t launch_wave(const WaveTables &t, const AdvanceArgs &a, bool fp32_lu, int waves_per_block,
                       int grid, hipStream_t stream);
// Zero n 64-bit words with a kernel (graph-capturable, unlike a memset node).
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t stream);
size_t wave_lds_bytes(const WaveTables &t, bool fp32_lu);

}  // namespace kin
