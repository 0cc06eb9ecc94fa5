// kin_xlane.h -- wavefront-level helpers shared by the table-driven kernels: a wavefront-local
// memory fence, scalar-loaded tables, DPP and readlane reductions, and the pivot search.
// Included inside namespace kin { namespace { ... } } of each kernel file.
#ifndef KIN_XLANE_H
#define KIN_XLANE_H

constexpr double kTmin = 200.0, kTmax = 6000.0;
constexpr int kW = 64;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Read-only tables indexed by wave-uniform values go through the constant address space,
// which lets the compiler use scalar loads for them.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *uniform_table(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}

// Diagnostic record of one cell's sub-step schedule (AdvanceArgs::trace), kept wave-uniform:
// the attempts' accept bits fill a 64-bit word that lane 0 stores when it is full, and the
// attempt count goes to word 0 at the end.  Inactive (p null) unless a trace was asked for.
struct ScheduleTrace {
    unsigned long long *p = nullptr;
    long long cap = 0, n = 0;
    unsigned long long w = 0;
    __device__ void start(unsigned long long *base, int words, long long g)
    {
        p = base ? base + (size_t)g * words : nullptr;
        cap = 64LL * (words - 1);
        n = 0;
        w = 0;
    }
    __device__ void add(bool accepted, int lane)
    {
        if (!p) return;
        if (n < cap) {
            w |= (unsigned long long)(accepted ? 1 : 0) << (n & 63);
            if ((n & 63) == 63) {
                if (lane == 0) p[1 + (n >> 6)] = w;
                w = 0;
            }
        }
        ++n;
    }
    __device__ void finish(int lane)
    {
        if (!p || lane != 0) return;
        const long long rec = n < cap ? n : cap;
        if (rec & 63) p[1 + (rec >> 6)] = w;
        p[0] = (unsigned long long)n;
    }
};

// ---- cross-lane helpers (all lanes of the wavefront must be active) ------------------------
template <int CTRL>
__device__ __forceinline__ int dpp(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp<CTRL>((int)b), hi = dpp<CTRL>((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(float, dpp<CTRL>(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ double rdlane(double v, int l)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float rdlane(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

constexpr int kLuBlock = 4;  // pivot steps between register rotations in the wave LU
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror: after the four
// steps every lane of a 16-lane row has combined all sixteen of the row's values.
constexpr int kDppX1 = 0xB1, kDppX2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// Wave-wide sum; every lane returns the same value.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp<kDppX1>(v);
    v += dpp<kDppX2>(v);
    v += dpp<kDppHalfMirror>(v);
    v += dpp<kDppMirror>(v);
    return (rdlane(v, 0) + rdlane(v, 16)) + (rdlane(v, 32) + rdlane(v, 48));
}

// Pivot search.  A non-negative floating-point value orders like its bit pattern read as an
// unsigned integer, so the largest |a_ik| is an integer maximum of those patterns (rows out of
// the search take key 0).  The lanes holding the maximum come from a ballot; when there are
// several (an exact tie), the one of lowest current row position wins.
template <int CTRL>
__device__ __forceinline__ unsigned dpp(unsigned v)
{
    return (unsigned)dpp<CTRL>((int)v);
}

__device__ __forceinline__ unsigned rdlane(unsigned v, int l) { return (unsigned)__builtin_amdgcn_readlane((int)v, l); }

template <typename K>
__device__ __forceinline__ K kmax(K a, K b) { return a > b ? a : b; }

// Wave-wide maximum; every lane returns the same value.
template <typename K>
__device__ __forceinline__ K wave_max(K v)
{
    v = kmax(v, dpp<kDppX1>(v));
    v = kmax(v, dpp<kDppX2>(v));
    v = kmax(v, dpp<kDppHalfMirror>(v));
    v = kmax(v, dpp<kDppMirror>(v));
    return kmax(kmax(rdlane(v, 0), rdlane(v, 16)), kmax(rdlane(v, 32), rdlane(v, 48)));
}

// Wave-wide minimum of non-negative ints; every lane returns the same value.
__device__ __forceinline__ int wave_min(int v)
{
    v = min(v, dpp<kDppX1>(v));
    v = min(v, dpp<kDppX2>(v));
    v = min(v, dpp<kDppHalfMirror>(v));
    v = min(v, dpp<kDppMirror>(v));
    return min(min(rdlane(v, 0), rdlane(v, 16)), min(rdlane(v, 32), rdlane(v, 48)));
}

// Lane holding the pivot row among lanes with `cand` set.  For doubles the maximum is taken
// over the high words first and, among lanes that tie there, over the low words: the same
// order as the full 64-bit keys, with 32-bit reductions that fuse with DPP.
template <typename R>
__device__ __forceinline__ int pivot_lane(R mag, bool cand, int pos)
{
    unsigned long long m;
    if constexpr (sizeof(R) == 8) {
        const unsigned long long k = cand ? __builtin_bit_cast(unsigned long long, mag) : 0ull;
        // the reductions run as statements of their own: inside a && they would run on the
        // candidate lanes only, and the cross-lane reads need every lane
        const unsigned hi = (unsigned)(k >> 32);
        const unsigned mh = wave_max(hi);
        m = __ballot(cand & (hi == mh));
        if (__builtin_popcountll(m) != 1) {
            const bool in = (m >> __lane_id()) & 1ull;
            const unsigned lo = in ? (unsigned)k : 0u;
            const unsigned ml = wave_max(lo);
            m = __ballot(in & (lo == ml));
        }
    } else {
        const unsigned k = cand ? __builtin_bit_cast(unsigned, mag) : 0u;
        const unsigned mk = wave_max(k);
        m = __ballot(cand & (k == mk));
    }
    if (__builtin_popcountll(m) == 1) return __builtin_ctzll(m);
    const int pmin = wave_min(((m >> __lane_id()) & 1ull) ? pos : 0x7fffffff);
    return __builtin_ctzll(__ballot(pos == pmin));
}


#endif
