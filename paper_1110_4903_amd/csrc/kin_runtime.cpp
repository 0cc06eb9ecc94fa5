// kin_runtime.cpp -- the C ABI of libkin: contexts, device-resident mechanisms and cell
// instances, advance launches, downloads.  See include/kin.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "kin_internal.h"

namespace kin {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

struct Mech {
    MechHost h;
    void *dbuf = nullptr;
    size_t dbytes = 0;
    WaveTables tab{};
    int layout = KIN_LAYOUT_WAVE;
    int block = 64;          // lane layout: threads per block; wave layout: waves per block
    hipModule_t mod = nullptr;
    hipFunction_t lane_f64 = nullptr, lane_f32 = nullptr, lane_cost = nullptr;
    // the same lane kernels compiled with the schedule recorder (kin_advance_trace only)
    hipModule_t mod_tr = nullptr;
    hipFunction_t lane_f64_tr = nullptr, lane_f32_tr = nullptr;
    int lane_block_tr = 0;
    double *kconst = nullptr;  // constant table of the lane kernels
    int lane_block = 0;      // block size the module was compiled for
    // autotuned (layout, block) per (precision, size class of the launch's cell count); a launch
    // of a class without an entry uses (layout, block) above
    std::map<std::pair<int, int>, std::pair<int, int>> tuned;
    double jit_seconds = 0.0;
    int refs = 0;
};

struct Inst {
    int mech = 0;
    long long n = 0, ld = 0;
    void *buf = nullptr;
    size_t bytes = 0;
    double *rho = nullptr, *e0 = nullptr, *T = nullptr, *Y = nullptr;
    int *status = nullptr, *level = nullptr, *iters = nullptr;
    unsigned long long *counter = nullptr;  // work counter of the advance kernels
    unsigned long long *sched = nullptr;    // per-cell sub-step schedule hash
    bool iters_current = false;  // iters[] holds the counts of an advance of the current state
};

// Instances at least this large take their cells in cost order: about four times the cells
// the layout keeps in flight (65536 lanes in the lane layout, a few thousand wavefronts in
// the others); below that every cell starts almost at once and the order only costs.
constexpr long long kOrderMinCells = 32768;
constexpr long long kOrderMinLaneCells = 262144;

// Code objects already compiled in this process, keyed by their source.
static std::mutex g_jit_mu;
static std::unordered_map<std::string, std::pair<std::vector<char>, double>> g_jit_cache;

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static uint64_t inst_bytes(int ns, long long n) { return (uint64_t)arena_bytes(n, ns); }

// A fluid grid: conserved state Q [ns + 3][ny][nx] and the workspace of its sweeps, one allocation.
struct Fluid {
    int mech = 0;
    FluidGrid g{};
    double dx = 0.0, dy = 0.0;
    void *buf = nullptr;
    double *Q = nullptr, *Q1 = nullptr, *W = nullptr, *T = nullptr, *F = nullptr, *KE = nullptr, *Es = nullptr;
    unsigned long long *speed = nullptr;
};

// A cached, instantiated graph of one batched advance.
struct Plan {
    hipGraphExec_t exec = nullptr;
    std::vector<int> insts;
    void *gwork = nullptr;  // workspace of the plan's global-layout launches (if any)
};

}  // namespace kin

struct kin_ctx {
    int device = 0;
    uint64_t budget = 0;
    uint64_t in_use = 0;
    int num_cu = 0;
    bool poisoned = false;
    std::string tune_cache;
    std::recursive_mutex mu;
    std::map<int, std::unique_ptr<kin::Mech>> mechs;
    std::map<int, std::unique_ptr<kin::Inst>> insts;
    std::map<int, std::unique_ptr<kin::Fluid>> fluids;
    int next_mech = 1, next_inst = 1, next_fluid = 1;
    // batched advances: capture streams (default priority), per-launch work counters and
    // instantiated graphs keyed by the launch description
    std::vector<hipStream_t> cap;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    unsigned long long *counters = nullptr;
    int ncounters = 0;
    std::map<std::string, kin::Plan> plans;
    kin_status plan_status = KIN_OK;
    // with a budget: one device pool of that size, carved first-fit into instance arenas
    char *pool = nullptr;
    // the device's fixed memory for kin_advance_noalloc (counters, then workspace)
    unsigned char *scratch = nullptr;
    // KIN_CTX_TIME_KERNELS: event pairs around advance kernels, the first kev_used recorded
    bool time_kernels = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> kev;
    size_t kev_used = 0;
    std::map<size_t, size_t> free_blocks;  // offset -> bytes, coalesced
};

using namespace kin;

// ---- instance memory: a first-fit pool when the context has a budget, else hipMalloc ----
static void *pool_alloc(kin_ctx *ctx, size_t bytes)
{
    for (auto it = ctx->free_blocks.begin(); it != ctx->free_blocks.end(); ++it) {
        if (it->second < bytes) continue;
        const size_t off = it->first, left = it->second - bytes;
        ctx->free_blocks.erase(it);
        if (left) ctx->free_blocks[off + bytes] = left;
        return ctx->pool + off;
    }
    return nullptr;
}

static void pool_free(kin_ctx *ctx, void *p, size_t bytes)
{
    size_t off = static_cast<char *>(p) - ctx->pool;
    auto next = ctx->free_blocks.lower_bound(off);
    if (next != ctx->free_blocks.end() && off + bytes == next->first) {
        bytes += next->second;
        next = ctx->free_blocks.erase(next);
    }
    if (next != ctx->free_blocks.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            prev->second += bytes;
            return;
        }
    }
    ctx->free_blocks[off] = bytes;
}

static size_t pool_largest(const kin_ctx *ctx)
{
    size_t m = 0;
    for (const auto &kv : ctx->free_blocks) m = std::max(m, kv.second);
    return m;
}

#define KIN_HIP(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            (ctx)->poisoned = true;                                                          \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));                    \
            return KIN_EDEVICE;                                                              \
        }                                                                                    \
    } while (0)

static kin_status err(kin_status s, const std::string &m)
{
    set_error(m);
    return s;
}

static kin_status enter(kin_ctx *ctx)
{
    if (!ctx) return err(KIN_EINVAL, "NULL context");
    if (ctx->poisoned) return err(KIN_EDEVICE, "context poisoned by an earlier device error");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return err(KIN_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    return KIN_OK;
}

extern "C" {

void kin_default_solver_opts(kin_solver_opts *s)
{
    if (!s) return;
    s->rtol = 1e-12;
    s->atol_Y = 1e-20;
    s->atol_T = 1e-9;
    s->y_neg = 1e-10;
    s->k_max = 10;
    s->L_max = 40;
    s->layout = KIN_LAYOUT_AUTO;
    s->L_forced = -1;
    s->max_iters = 100000;
    s->point_implicit = 0;
    s->diverge_ratio = 2.0;
}

const char *kin_last_error(void) { return g_err.c_str(); }

kin_status kin_create(kin_ctx **out, const kin_ctx_opts *o)
{
    if (!out) return err(KIN_EINVAL, "NULL output pointer");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return err(KIN_EDEVICE, "no HIP device available");
    std::unique_ptr<kin_ctx> c(new kin_ctx());
    c->device = o ? o->device : 0;
    if (c->device < 0 || c->device >= ndev) return err(KIN_EINVAL, "device ordinal out of range");
    c->budget = o ? o->hbm_budget : 0;
    c->time_kernels = o && (o->flags & KIN_CTX_TIME_KERNELS);
    if (o && o->tune_cache) c->tune_cache = o->tune_cache;
    else if (const char *env = std::getenv("KIN_TUNE_CACHE")) c->tune_cache = env;
    if ((e = hipSetDevice(c->device)) != hipSuccess) return err(KIN_EDEVICE, hipGetErrorString(e));
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, c->device)) != hipSuccess) return err(KIN_EDEVICE, hipGetErrorString(e));
    c->num_cu = prop.multiProcessorCount;
    // address of this device's fixed memory for the allocation-free advance (once per device)
    if ((e = scratch_address(c->device, &c->scratch)) != hipSuccess)
        return err(KIN_EDEVICE, std::string("fixed device memory: ") + hipGetErrorString(e));
    if (c->budget) {
        c->budget &= ~(uint64_t)255;
        if (c->budget == 0) return err(KIN_EINVAL, "budget below 256 bytes");
        if ((e = hipMalloc(reinterpret_cast<void **>(&c->pool), c->budget)) != hipSuccess)
            return err(KIN_ENOMEM, std::string("cannot reserve the budget: ") + hipGetErrorString(e));
        c->free_blocks[0] = c->budget;
    }
    *out = c.release();
    return KIN_OK;
}

void kin_destroy(kin_ctx *ctx)
{
    if (!ctx) return;
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        hipSetDevice(ctx->device);
        hipDeviceSynchronize();
        for (auto &kv : ctx->plans) {
            hipGraphExecDestroy(kv.second.exec);
            if (kv.second.gwork) hipFree(kv.second.gwork);
        }
        for (hipStream_t st : ctx->cap) hipStreamDestroy(st);
        for (hipEvent_t ev : ctx->join) hipEventDestroy(ev);
        for (auto &p : ctx->kev) {
            hipEventDestroy(p.first);
            hipEventDestroy(p.second);
        }
        if (ctx->fork) hipEventDestroy(ctx->fork);
        hipFree(ctx->counters);
        for (auto &kv : ctx->fluids) hipFree(kv.second->buf);
        if (ctx->pool) hipFree(ctx->pool);
        else
            for (auto &kv : ctx->insts) hipFree(kv.second->buf);
        for (auto &kv : ctx->mechs) {
            if (kv.second->mod) hipModuleUnload(kv.second->mod);
            if (kv.second->mod_tr) hipModuleUnload(kv.second->mod_tr);
            hipFree(kv.second->dbuf);
            hipFree(kv.second->kconst);
        }
    }
    delete ctx;
}

// Lane-layout kernels of a mechanism, compiled for the given block size.
static kin_status build_lane(kin_ctx *ctx, Mech &m, int block)
{
    if (m.mod && m.lane_block == block) return KIN_OK;
    std::vector<double> consts;
    const std::string src = lane_source(m.h, block, consts);
    std::vector<char> code;
    double secs = 0.0;
    {
        std::lock_guard<std::mutex> lk(g_jit_mu);
        auto it = g_jit_cache.find(src);
        if (it != g_jit_cache.end()) {
            code = it->second.first;
        } else {
            std::string msg;
            kin_status s = rtc_compile(src, "kin_lane.hip", code, msg, &secs);
            if (s != KIN_OK) return err(s, msg);
            g_jit_cache.emplace(src, std::make_pair(code, secs));
        }
    }
    if (m.mod) {
        hipModuleUnload(m.mod);
        m.mod = nullptr;
    }
    if (!m.kconst) {
        KIN_HIP(ctx, hipMalloc(&m.kconst, sizeof(double) * std::max<size_t>(consts.size(), 1)));
        if (!consts.empty())
            KIN_HIP(ctx, hipMemcpy(m.kconst, consts.data(), sizeof(double) * consts.size(), hipMemcpyHostToDevice));
    }
    KIN_HIP(ctx, hipModuleLoadData(&m.mod, code.data()));
    KIN_HIP(ctx, hipModuleGetFunction(&m.lane_f64, m.mod, "kin_lane_f64"));
    KIN_HIP(ctx, hipModuleGetFunction(&m.lane_f32, m.mod, "kin_lane_f32lu"));
    KIN_HIP(ctx, hipModuleGetFunction(&m.lane_cost, m.mod, "kin_lane_cost"));
    m.lane_block = block;
    m.jit_seconds += secs;
    return KIN_OK;
}

// Lane-layout kernels with the schedule recorder (KIN_TRACE), compiled on first use.
static kin_status build_lane_trace(kin_ctx *ctx, Mech &m, int block)
{
    if (m.mod_tr && m.lane_block_tr == block) return KIN_OK;
    kin_status s = build_lane(ctx, m, block);  // the constant table
    if (s != KIN_OK) return s;
    std::vector<double> consts;
    const std::string src = "#define KIN_TRACE 1\n" + lane_source(m.h, block, consts);
    std::vector<char> code;
    {
        std::lock_guard<std::mutex> lk(g_jit_mu);
        auto it = g_jit_cache.find(src);
        if (it != g_jit_cache.end()) {
            code = it->second.first;
        } else {
            std::string msg;
            double secs = 0.0;
            if ((s = rtc_compile(src, "kin_lane_trace.hip", code, msg, &secs)) != KIN_OK) return err(s, msg);
            g_jit_cache.emplace(src, std::make_pair(code, secs));
        }
    }
    if (m.mod_tr) {
        hipModuleUnload(m.mod_tr);
        m.mod_tr = nullptr;
    }
    KIN_HIP(ctx, hipModuleLoadData(&m.mod_tr, code.data()));
    KIN_HIP(ctx, hipModuleGetFunction(&m.lane_f64_tr, m.mod_tr, "kin_lane_f64"));
    KIN_HIP(ctx, hipModuleGetFunction(&m.lane_f32_tr, m.mod_tr, "kin_lane_f32lu"));
    m.lane_block_tr = block;
    return KIN_OK;
}

// Pack the device tables of the table-driven kernels.
static kin_status upload_tables(kin_ctx *ctx, Mech &m)
{
    const MechHost &h = m.h;
    const int ns = h.ns, nr = h.nr;
    const int nchunk = (nr + kChunk - 1) / kChunk;
    // third-body reactions get slots of their own (two reactions may share an efficiency row)
    std::vector<int> slot(nr, -1), slot_row;
    for (int r = 0; r < nr; ++r)
        if (h.rx[r].tb >= 0) {
            slot[r] = (int)slot_row.size();
            slot_row.push_back(h.rx[r].tb);
        }
    const int ntb = (int)slot_row.size();
    // reactions in order of (reactant count, product count), so that each pass of 64 lanes is
    // homogeneous and its loops over slots stop at the pass's largest counts
    const int npad = wave_npad(ns + 1);
    // for the wave layout's dense third-body product: slots whose reaction has a participant in
    // the last 16-row tile come first, so that the tile's product stops after their steps
    int tb_last = ntb;
    if (npad > 0 && ntb > 0) {
        const int row0 = 16 * ((npad + 15) / 16 - 1);
        std::vector<char> touch(ntb, 0);
        for (int r = 0; r < nr; ++r) {
            if (slot[r] < 0) continue;
            const Rxn &x = h.rx[r];
            for (int j = 0; j < x.npart; ++j)
                if (x.part[j].nu && x.part[j].sp >= row0) touch[slot[r]] = 1;
        }
        std::vector<int> renum(ntb), order;
        for (int q = 0; q < ntb; ++q) if (touch[q]) order.push_back(q);
        tb_last = (int)order.size();
        for (int q = 0; q < ntb; ++q) if (!touch[q]) order.push_back(q);
        std::vector<int> row_new(ntb);
        for (int i = 0; i < ntb; ++i) { renum[order[i]] = i; row_new[i] = slot_row[order[i]]; }
        for (int r = 0; r < nr; ++r) if (slot[r] >= 0) slot[r] = renum[slot[r]];
        slot_row.swap(row_new);
    }
    std::vector<int> perm(nr);
    for (int r = 0; r < nr; ++r) perm[r] = r;
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
        const Rxn &x = h.rx[a], &y = h.rx[b];
        return x.nreac != y.nreac ? x.nreac < y.nreac : x.nprod < y.nprod;
    });
    std::vector<int> chunk_rp(nchunk, 0);
    for (int i = 0; i < nr; ++i) {
        const Rxn &x = h.rx[perm[i]];
        int &c = chunk_rp[i / kChunk];
        c = std::max(c & 0xff, x.nreac) | (std::max(c >> 8, x.nprod) << 8);
    }
    std::vector<double> rxd((size_t)nr * 4);
    std::vector<RxnRec> rxc(nr);
    std::vector<RxnCoef> rxk(nr);
    for (int i = 0; i < nr; ++i) {
        const int r = perm[i];
        const Rxn &x = h.rx[r];
        rxd[4 * i + 0] = x.lnA;
        rxd[4 * i + 1] = x.b;
        rxd[4 * i + 2] = x.Ta;
        rxd[4 * i + 3] = (double)x.dnu;
        RxnRec &p = rxc[i];
        RxnCoef &k = rxk[i];
        std::memset(&p, 0, sizeof p);
        std::memset(&k, 0, sizeof k);
        p.rev = (int8_t)x.rev;
        p.tb = (int16_t)slot[r];
        for (int m = 0; m < 3; ++m) {
            for (int side = 0; side < 2; ++side) {
                const int n = side ? x.nprod : x.nreac;
                if (m >= n) continue;
                const int sp = side ? x.prod_sp[m] : x.reac_sp[m];
                const int nu = side ? x.prod_nu[m] : -x.reac_nu[m];
                const int q = 3 * side + m;
                p.nu[q] = (int8_t)nu;
                p.coff[q] = (uint16_t)(8 * sp);
                p.roff[q] = (uint16_t)(npad > 0 ? 8 * sp * (npad + 1) : 0);  // wave layout only (row stride NPAD + 1)
                k.rowc[q] = (double)nu * h.M[sp];
                k.colc[q] = 1.0 / h.M[sp];
            }
        }
    }
    // e_s(T_ref) at T_ref = 298.15 K (J/kg) for the conserved-variable adapter
    std::vector<double> ef(ns);
    for (int s = 0; s < ns; ++s) {
        const double Tr = 298.15;
        const double *a = &h.nasa[(size_t)14 * s + (Tr < h.Tmid[s] ? 0 : 7)];
        const double h_RT = a[0] + Tr * (a[1] / 2 + Tr * (a[2] / 3 + Tr * (a[3] / 4 + Tr * a[4] / 5))) + a[5] / Tr;
        ef[s] = 8.31446261815324e3 / h.M[s] * Tr * (h_RT - 1.0);
    }
    // dense third-body terms as a small matrix product per cell: J[s][k] += sum_q A[s][q] B[q][k]
    // with A[s][q] = nu_qs M_s D_q (D_q = q_f - q_b of slot q, known only in the kernel) and
    // B[q][k] = eff_qk / M_k.  tbA holds nu_qs M_s and tbB holds B, both cut into the operand
    // tiles of the 16x16x4 matrix instruction: tile (kk, t) is 64 values, lane l of tbA's tile
    // holding row 16 t + l % 16 and slot 4 kk + l / 16, lane l of tbB's tile holding slot
    // 4 kk + l / 16 and column 16 t + l % 16.  There are ceil(NPAD / 16) row tiles (NPAD the
    // wave layout's padded row length) and slot steps in whole groups of four; entries outside
    // the mechanism are zero.
    std::vector<double> effT((size_t)std::max(1, ns * ntb), 0.0);
    std::vector<double> nuM((size_t)ns * std::max(1, ntb), 0.0);
    int ntbe = 0;
    for (int r = 0; r < nr; ++r) {
        const int q = slot[r];
        if (q < 0) continue;
        const Rxn &x = h.rx[r];
        for (int j = 0; j < x.npart; ++j) {
            if (!x.part[j].nu) continue;
            const int s = x.part[j].sp;
            nuM[(size_t)s * ntb + q] += (double)x.part[j].nu * h.M[s];
            ++ntbe;
        }
    }
    // (only the wave layout reads them: mechanisms too large for it get empty tables)
    const int tb_nt = npad > 0 ? (npad + 15) / 16 : 0, tb_nk = npad > 0 ? 4 * ((ntb + 15) / 16) : 0;
    std::vector<double> tbA((size_t)std::max(1, tb_nk * tb_nt) * 64, 0.0), tbB(tbA.size(), 0.0);
    for (int kk = 0; kk < tb_nk; ++kk)
        for (int ti = 0; ti < tb_nt; ++ti)
            for (int l = 0; l < 64; ++l) {
                const int q = 4 * kk + l / 16, rc = 16 * ti + l % 16;
                if (q >= ntb || rc >= ns) continue;
                const size_t o = ((size_t)kk * tb_nt + ti) * 64 + l;
                tbA[o] = nuM[(size_t)rc * ntb + q];
                tbB[o] = h.eff[(size_t)slot_row[q] * ns + rc] / h.M[rc];
            }
    for (int r = 0; r < nr; ++r) {
        const int q = slot[r];
        if (q < 0) continue;
        for (int k = 0; k < ns; ++k) effT[(size_t)k * ntb + q] = h.eff[(size_t)slot_row[q] * ns + k];
    }
    std::vector<double> effTM(effT);
    for (int k = 0; k < ns; ++k)
        for (int q = 0; q < ntb; ++q) effTM[(size_t)k * ntb + q] /= h.M[k];
    // the same entries ordered by slot, with their row factors (global-memory layout: one
    // pass of lanes over entries adds into distinct rows)
    std::vector<int> tgs;
    std::vector<double> tgf;
    for (int r = 0; r < nr; ++r) {
        const int q = slot[r];
        if (q < 0) continue;
        const Rxn &x = h.rx[r];
        for (int s = 0; s < ns; ++s)
            for (int j = 0; j < x.npart; ++j) {
                if (!x.part[j].nu || x.part[j].sp != s) continue;
                tgs.push_back(q | (s << 16));
                tgf.push_back((double)x.part[j].nu * h.M[s]);
            }
    }
    if (tgs.empty()) { tgs.push_back(0); tgf.push_back(0.0); }
    // one allocation, 256-byte aligned pieces
    struct Piece { const void *src; size_t bytes; size_t off; };
    std::vector<Piece> pc = {
        {h.nasa.data(), sizeof(double) * h.nasa.size(), 0}, {h.Tmid.data(), sizeof(double) * ns, 0},
        {h.M.data(), sizeof(double) * ns, 0}, {rxd.data(), sizeof(double) * rxd.size(), 0},
        {rxc.data(), sizeof(RxnRec) * rxc.size(), 0}, {rxk.data(), sizeof(RxnCoef) * rxk.size(), 0},
        {effT.data(), sizeof(double) * effT.size(), 0}, {tbA.data(), sizeof(double) * tbA.size(), 0},
        {tbB.data(), sizeof(double) * tbB.size(), 0}, {chunk_rp.data(), sizeof(int) * chunk_rp.size(), 0},
        {ef.data(), sizeof(double) * ns, 0}, {tgs.data(), sizeof(int) * tgs.size(), 0},
        {tgf.data(), sizeof(double) * tgf.size(), 0}, {effTM.data(), sizeof(double) * effTM.size(), 0}};
    size_t total = 0;
    for (Piece &p : pc) { p.off = total; total = align256(total + p.bytes); }
    std::vector<char> host(total, 0);
    for (const Piece &p : pc) std::memcpy(&host[p.off], p.src, p.bytes);
    KIN_HIP(ctx, hipMalloc(&m.dbuf, total));
    m.dbytes = total;
    KIN_HIP(ctx, hipMemcpy(m.dbuf, host.data(), total, hipMemcpyHostToDevice));
    char *b = static_cast<char *>(m.dbuf);
    WaveTables &t = m.tab;
    t.ns = ns; t.nr = nr; t.ntb = ntb; t.nchunk = nchunk; t.ntbe = ntbe;
    t.tb_last = tb_last;
    t.lnPaR = std::log(kPatmCgs / kRuCgs);
    t.nasa = reinterpret_cast<const double *>(b + pc[0].off);
    t.Tmid = reinterpret_cast<const double *>(b + pc[1].off);
    t.M = reinterpret_cast<const double *>(b + pc[2].off);
    t.rxd = reinterpret_cast<const double *>(b + pc[3].off);
    t.rxc = reinterpret_cast<const RxnRec *>(b + pc[4].off);
    t.rxk = reinterpret_cast<const RxnCoef *>(b + pc[5].off);
    t.effT = reinterpret_cast<const double *>(b + pc[6].off);
    t.tbA = reinterpret_cast<const double *>(b + pc[7].off);
    t.tbB = reinterpret_cast<const double *>(b + pc[8].off);
    t.chunk_rp = reinterpret_cast<const int *>(b + pc[9].off);
    t.ef = reinterpret_cast<const double *>(b + pc[10].off);
    t.tgs = reinterpret_cast<const int *>(b + pc[11].off);
    t.tgf = reinterpret_cast<const double *>(b + pc[12].off);
    t.effTM = reinterpret_cast<const double *>(b + pc[13].off);
    return KIN_OK;
}

// ---- autotuner cache ----------------------------------------------------------------------
static uint64_t fnv(uint64_t h, const void *p, size_t n)
{
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
    return h;
}

static std::string tune_key(const kin_ctx *ctx, const Mech &m, int prec)
{
    uint64_t h = 0xcbf29ce484222325ull;
    const MechHost &x = m.h;
    h = fnv(h, &x.ns, sizeof x.ns);
    h = fnv(h, &x.nr, sizeof x.nr);
    h = fnv(h, x.M.data(), sizeof(double) * x.M.size());
    h = fnv(h, x.nasa.data(), sizeof(double) * x.nasa.size());
    for (const Rxn &r : x.rx) h = fnv(h, &r, sizeof r);
    h = fnv(h, x.eff.data(), sizeof(double) * x.eff.size());
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) h = fnv(h, prop.gcnArchName, std::strlen(prop.gcnArchName));
    char buf[64];
    std::snprintf(buf, sizeof buf, "%016llx-p%d", (unsigned long long)h, prec);
    return buf;
}

// The cache file holds one flat JSON object: {"<key>": [layout, block, ms], ...}.
static std::map<std::string, std::vector<double>> tune_read(const std::string &path)
{
    std::map<std::string, std::vector<double>> out;
    FILE *f = path.empty() ? nullptr : std::fopen(path.c_str(), "r");
    if (!f) return out;
    std::string txt;
    char buf[4096];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, r);
    std::fclose(f);
    size_t p = 0;
    while ((p = txt.find('"', p)) != std::string::npos) {
        const size_t q = txt.find('"', p + 1);
        if (q == std::string::npos) break;
        const std::string key = txt.substr(p + 1, q - p - 1);
        const size_t lb = txt.find('[', q), rb = txt.find(']', q);
        if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
        std::vector<double> v;
        std::string body = txt.substr(lb + 1, rb - lb - 1);
        size_t s0 = 0;
        while (s0 < body.size()) {
            size_t e = body.find(',', s0);
            if (e == std::string::npos) e = body.size();
            v.push_back(std::atof(body.substr(s0, e - s0).c_str()));
            s0 = e + 1;
        }
        out[key] = v;
        p = rb + 1;
    }
    return out;
}

static void tune_write(const std::string &path, const std::map<std::string, std::vector<double>> &m)
{
    if (path.empty()) return;
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m) {
        std::fprintf(f, "  \"%s\": [%d, %d, %.6g]%s\n", kv.first.c_str(), (int)kv.second[0], (int)kv.second[1],
                     kv.second.size() > 2 ? kv.second[2] : 0.0, ++i < m.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path.c_str());
}

kin_status kin_mech_upload(kin_ctx *ctx, const kin_mech_desc *d, int32_t *mech_id)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!mech_id) return err(KIN_EINVAL, "NULL mech_id");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    std::unique_ptr<Mech> m(new Mech());
    std::string msg;
    if ((s = mech_from_desc(d, m->h, msg)) != KIN_OK) return err(s, msg);
    if ((s = upload_tables(ctx, *m)) != KIN_OK) {
        hipFree(m->dbuf);
        return s;
    }
    if (m->h.ns <= kLaneNsMax) {
        m->layout = KIN_LAYOUT_LANE;
        m->block = 64;
        if ((s = build_lane(ctx, *m, m->block)) != KIN_OK) {
            hipFree(m->dbuf);
            hipFree(m->kconst);
            return s;
        }
    } else if (m->h.ns <= kWaveNsMax) {
        m->layout = KIN_LAYOUT_WAVE;
        m->block = 1;
    } else {
        m->layout = KIN_LAYOUT_GLOBAL;
        m->block = 64;
    }
    {   // tuned choices from the cache file, if any: per (precision, size class) ...
        const auto cache = tune_read(ctx->tune_cache);
        for (int prec : {(int)KIN_FP64, (int)KIN_FP32_LU})
            for (int c = 0; c <= 4; ++c) {
                auto it = cache.find(tune_key(ctx, *m, prec) + "-c" + std::to_string(c));
                if (it == cache.end() || it->second.size() < 2) continue;
                const int lay = (int)it->second[0], blk = (int)it->second[1];
                const bool ok = (lay == KIN_LAYOUT_WAVE && blk >= 1 && blk <= 4 && m->h.ns <= kWaveNsMax) ||
                                (lay == KIN_LAYOUT_LANE && lane_block_ok(m->h.ns, blk)) ||
                                (lay == KIN_LAYOUT_GLOBAL && blk == 64);
                if (ok) m->tuned[{prec, c}] = {lay, blk};
            }
        // ... and a mechanism-wide FP64 entry of an earlier cache format
        auto it = cache.find(tune_key(ctx, *m, KIN_FP64));
        if (it != cache.end() && it->second.size() >= 2) {
            const int lay = (int)it->second[0], blk = (int)it->second[1];
            if (lay == KIN_LAYOUT_WAVE && blk >= 1 && blk <= 4 && m->h.ns <= kWaveNsMax) {
                m->layout = lay;
                m->block = blk;
            } else if (lay == KIN_LAYOUT_LANE && m->h.ns <= kLaneNsMax && (blk == 64 || blk == 128 || blk == 256)) {
                if ((s = build_lane(ctx, *m, blk)) == KIN_OK) {
                    m->layout = lay;
                    m->block = blk;
                }
            }
        }
    }
    const int id = ctx->next_mech++;
    ctx->mechs[id] = std::move(m);
    *mech_id = id;
    return KIN_OK;
}

kin_status kin_mech_release(kin_ctx *ctx, int32_t mech_id)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->mechs.find(mech_id);
    if (it == ctx->mechs.end()) return err(KIN_ENOTFOUND, "unknown mechanism id");
    if (it->second->refs > 0) return err(KIN_EBUSY, "mechanism still used by instances");
    if (it->second->mod) hipModuleUnload(it->second->mod);
    if (it->second->mod_tr) hipModuleUnload(it->second->mod_tr);
    KIN_HIP(ctx, hipFree(it->second->dbuf));
    KIN_HIP(ctx, hipFree(it->second->kconst));
    ctx->mechs.erase(it);
    return KIN_OK;
}

kin_status kin_set_layout(kin_ctx *ctx, int32_t mech_id, int32_t layout, int32_t block)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->mechs.find(mech_id);
    if (it == ctx->mechs.end()) return err(KIN_ENOTFOUND, "unknown mechanism id");
    Mech &m = *it->second;
    if (layout == KIN_LAYOUT_LANE) {
        if (m.h.ns > kLaneNsMax) return err(KIN_EINVAL, "lane layout needs ns <= 15");
        if (!lane_block_ok(m.h.ns, block))
            return err(KIN_EINVAL, "lane block must be 64, 128 or 256 threads within 64 KiB of LDS for this mechanism");
        if ((s = build_lane(ctx, m, block)) != KIN_OK) return s;
    } else if (layout == KIN_LAYOUT_WAVE) {
        if (m.h.ns > kWaveNsMax) return err(KIN_EINVAL, "wave layout needs ns <= 63");
        if (block < 1 || block > 4) return err(KIN_EINVAL, "wave layout takes 1..4 wavefronts per block");
        if (wave_lds_bytes(m.tab, false) * (size_t)block > 65536)
            return err(KIN_EINVAL, "that many wavefronts per block exceed 64 KiB of LDS for this mechanism");
    } else if (layout == KIN_LAYOUT_GLOBAL) {
        if (block != 64) return err(KIN_EINVAL, "global layout runs 64 threads per block");
    } else {
        return err(KIN_EINVAL, "layout must be LANE, WAVE or GLOBAL");
    }
    m.layout = layout;
    m.block = block;
    m.tuned.clear();  // an explicit choice replaces the autotuned ones
    return KIN_OK;
}

static kin_status copy_in(kin_ctx *ctx, void *dst, const void *src, size_t bytes, kin_mem where,
                          hipStream_t st)
{
    if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    else if (where == KIN_MEM_PINNED) KIN_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    else KIN_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
    return KIN_OK;
}

static bool mem_ok(kin_mem w) { return w == KIN_MEM_HOST || w == KIN_MEM_DEVICE || w == KIN_MEM_PINNED; }

static hipMemcpyKind out_kind(kin_mem w)
{
    return w == KIN_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

static kin_status fill_state(kin_ctx *ctx, Inst &in, const Mech &m, const double *rho,
                             const double *T, const double *Y, const double *e0, kin_mem where,
                             hipStream_t st)
{
    const size_t nb = sizeof(double) * (size_t)in.n;
    kin_status s;
    if ((s = copy_in(ctx, in.rho, rho, nb, where, st)) != KIN_OK) return s;
    if ((s = copy_in(ctx, in.T, T, nb, where, st)) != KIN_OK) return s;
    if ((s = copy_in(ctx, in.Y, Y, nb * m.h.ns, where, st)) != KIN_OK) return s;
    if (e0) {
        if ((s = copy_in(ctx, in.e0, e0, nb, where, st)) != KIN_OK) return s;
    } else {
        KIN_HIP(ctx, launch_energy(m.tab, in.n, in.ld, in.T, in.Y, in.e0, st));
        if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipStreamSynchronize(st));
    }
    return KIN_OK;
}

// An instance's arena: from the budget pool when the context has one, else its own hipMalloc.
static kin_status alloc_inst(kin_ctx *ctx, int32_t mech_id, const Mech &m, int64_t n_cells,
                             std::unique_ptr<Inst> &out)
{
    const uint64_t bytes = inst_bytes(m.h.ns, n_cells);
    if (ctx->budget && ctx->in_use + bytes > ctx->budget)
        return err(KIN_ENOMEM, "instance of " + std::to_string(bytes) + " bytes exceeds the context budget");
    std::unique_ptr<Inst> in(new Inst());
    in->mech = mech_id;
    in->n = n_cells;
    in->ld = n_cells;
    in->bytes = bytes;
    if (ctx->pool) {
        if (!(in->buf = pool_alloc(ctx, bytes)))
            return err(KIN_ENOMEM, "no free block of " + std::to_string(bytes) + " bytes in the budget");
    } else {
        KIN_HIP(ctx, hipMalloc(&in->buf, bytes));
    }
    const Arena ar = arena_at(static_cast<char *>(in->buf), n_cells, m.h.ns);
    in->rho = ar.rho; in->e0 = ar.e0; in->T = ar.T; in->Y = ar.Y; in->sched = ar.sched;
    in->status = ar.status; in->level = ar.level; in->iters = ar.iters; in->counter = ar.counter;
    out = std::move(in);
    return KIN_OK;
}

static void free_inst_buf(kin_ctx *ctx, Inst &in)
{
    if (ctx->pool) pool_free(ctx, in.buf, in.bytes);
    else hipFree(in.buf);
}

// Conserved state into an instance's arena: rho_s goes into the Y slot, E_sens into e0 and the
// start temperatures into T, and the conversion kernel rewrites them in place.
static kin_status fill_conserved(kin_ctx *ctx, Inst &in, const Mech &m, const double *rho_s,
                                 const double *E_sens, const double *T_guess, kin_mem where,
                                 hipStream_t st)
{
    const size_t nb = sizeof(double) * (size_t)in.n;
    kin_status s;
    if ((s = copy_in(ctx, in.Y, rho_s, nb * m.h.ns, where, st)) != KIN_OK) return s;
    if ((s = copy_in(ctx, in.e0, E_sens, nb, where, st)) != KIN_OK) return s;
    if (T_guess && (s = copy_in(ctx, in.T, T_guess, nb, where, st)) != KIN_OK) return s;
    KIN_HIP(ctx, launch_conserved_in(m.tab, in.n, in.ld, in.rho, in.T, in.Y, in.e0, T_guess != nullptr, st));
    return KIN_OK;
}

// Clear the per-cell diagnostics and register a filled instance.
static kin_status commit_inst(kin_ctx *ctx, Mech &m, std::unique_ptr<Inst> &in, kin_mem where,
                              hipStream_t st, int32_t *inst_id)
{
    const size_t i = align256(sizeof(int) * (size_t)in->n);
    KIN_HIP(ctx, hipMemsetAsync(in->status, 0, 3 * i, st));
    if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipStreamSynchronize(st));
    m.refs++;
    ctx->in_use += in->bytes;
    const int id = ctx->next_inst++;
    ctx->insts[id] = std::move(in);
    *inst_id = id;
    return KIN_OK;
}

kin_status kin_state_upload(kin_ctx *ctx, int32_t mech_id, int64_t n_cells, const double *rho,
                            const double *T, const double *Y, const double *e0, kin_mem where,
                            void *stream, int32_t *inst_id)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!inst_id || n_cells < 1 || !rho || !T || !Y) return err(KIN_EINVAL, "bad state arguments");
    if (!mem_ok(where)) return err(KIN_EINVAL, "bad memory kind");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->mechs.find(mech_id);
    if (it == ctx->mechs.end()) return err(KIN_ENOTFOUND, "unknown mechanism id");
    Mech &m = *it->second;
    std::unique_ptr<Inst> in;
    if ((s = alloc_inst(ctx, mech_id, m, n_cells, in)) != KIN_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((s = fill_state(ctx, *in, m, rho, T, Y, e0, where, st)) != KIN_OK) {
        free_inst_buf(ctx, *in);
        return s;
    }
    return commit_inst(ctx, m, in, where, st, inst_id);
}

kin_status kin_state_upload_conserved(kin_ctx *ctx, int32_t mech_id, int64_t n_cells,
                                      const double *rho_s, const double *E_sens,
                                      const double *T_guess, kin_mem where, void *stream,
                                      int32_t *inst_id)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!inst_id || n_cells < 1 || !rho_s || !E_sens) return err(KIN_EINVAL, "bad conserved-state arguments");
    if (!mem_ok(where)) return err(KIN_EINVAL, "bad memory kind");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->mechs.find(mech_id);
    if (it == ctx->mechs.end()) return err(KIN_ENOTFOUND, "unknown mechanism id");
    Mech &m = *it->second;
    std::unique_ptr<Inst> in;
    if ((s = alloc_inst(ctx, mech_id, m, n_cells, in)) != KIN_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((s = fill_conserved(ctx, *in, m, rho_s, E_sens, T_guess, where, st)) != KIN_OK) {
        free_inst_buf(ctx, *in);
        return s;
    }
    return commit_inst(ctx, m, in, where, st, inst_id);
}

kin_status kin_state_reset_conserved(kin_ctx *ctx, int32_t inst_id, const double *rho_s,
                                     const double *E_sens, const double *T_guess, kin_mem where,
                                     void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!rho_s || !E_sens) return err(KIN_EINVAL, "NULL conserved-state array");
    if (!mem_ok(where)) return err(KIN_EINVAL, "bad memory kind");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->insts.find(inst_id);
    if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
    Inst &in = *it->second;
    const Mech &m = *ctx->mechs[in.mech];
    hipStream_t st = static_cast<hipStream_t>(stream);
    in.iters_current = false;
    if ((s = fill_conserved(ctx, in, m, rho_s, E_sens, T_guess, where, st)) != KIN_OK) return s;
    if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipStreamSynchronize(st));
    return KIN_OK;
}

kin_status kin_download_conserved(kin_ctx *ctx, int32_t inst_id, double *rho_s, double *E_sens,
                                  kin_mem where, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!rho_s || !E_sens) return err(KIN_EINVAL, "NULL destination");
    if (!mem_ok(where)) return err(KIN_EINVAL, "bad memory kind");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->insts.find(inst_id);
    if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
    const Inst &in = *it->second;
    const Mech &m = *ctx->mechs[in.mech];
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (where == KIN_MEM_DEVICE) {
        KIN_HIP(ctx, launch_conserved_out(m.tab, in.n, in.ld, in.rho, in.Y, in.e0, rho_s, E_sens, st));
        return KIN_OK;
    }
    const size_t nb = sizeof(double) * (size_t)in.n;
    double *stage = nullptr;
    KIN_HIP(ctx, hipMallocAsync(reinterpret_cast<void **>(&stage), nb * (m.h.ns + 1), st));
    KIN_HIP(ctx, launch_conserved_out(m.tab, in.n, in.ld, in.rho, in.Y, in.e0, stage, stage + (size_t)in.n * m.h.ns, st));
    KIN_HIP(ctx, hipMemcpyAsync(rho_s, stage, nb * m.h.ns, hipMemcpyDeviceToHost, st));
    KIN_HIP(ctx, hipMemcpyAsync(E_sens, stage + (size_t)in.n * m.h.ns, nb, hipMemcpyDeviceToHost, st));
    KIN_HIP(ctx, hipFreeAsync(stage, st));
    if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipStreamSynchronize(st));
    return KIN_OK;
}

kin_status kin_state_reset(kin_ctx *ctx, int32_t inst_id, const double *rho, const double *T,
                           const double *Y, const double *e0, kin_mem where, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!rho || !T || !Y) return err(KIN_EINVAL, "NULL state array");
    if (!mem_ok(where)) return err(KIN_EINVAL, "bad memory kind");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->insts.find(inst_id);
    if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
    Inst &in = *it->second;
    const Mech &m = *ctx->mechs[in.mech];
    in.iters_current = false;
    return fill_state(ctx, in, m, rho, T, Y, e0, where, static_cast<hipStream_t>(stream));
}

static void fill_opts(AdvanceArgs &a, const kin_solver_opts &o)
{
    a.rtol = o.rtol; a.atol_Y = o.atol_Y; a.atol_T = o.atol_T; a.y_neg = o.y_neg;
    a.k_max = o.k_max; a.L_max = o.L_max; a.L_forced = o.L_forced; a.max_iters = o.max_iters;
    a.point_implicit = o.point_implicit ? 1 : 0;
    a.diverge_ratio = o.diverge_ratio;
    if (a.point_implicit) {  // one sub-step over dt, one (linearised) update
        a.L_forced = 0;
        a.k_max = 1;
    }
}

// Size class of a launch's cell count for the autotuner: below 4096, 16384, 65536, 262144, and
// the rest.  A lane-layout launch fills the device's 65536 lanes only from the top class on,
// so small launches can prefer another layout.
static int size_class(long long cells)
{
    return cells < 4096 ? 0 : cells < 16384 ? 1 : cells < 65536 ? 2 : cells < 262144 ? 3 : 4;
}

// Effective (layout, block) of a mechanism for these options and a launch of `cells` cells:
// an explicit layout in the options, else the autotuned choice for the launch's size class and
// precision, else the mechanism's layout.
static void layout_of(const Mech &m, const kin_solver_opts &o, int prec, long long cells, int &layout, int &block)
{
    if (o.layout == KIN_LAYOUT_AUTO) {
        auto it = m.tuned.find({prec, size_class(cells)});
        if (it != m.tuned.end()) {
            layout = it->second.first;
            block = it->second.second;
            return;
        }
    }
    layout = o.layout == KIN_LAYOUT_AUTO ? m.layout : o.layout;
    if (layout == KIN_LAYOUT_LANE) block = (m.layout == KIN_LAYOUT_LANE) ? m.block : 64;
    else if (layout == KIN_LAYOUT_WAVE) block = (m.layout == KIN_LAYOUT_WAVE) ? m.block : 1;
    else block = 64;
}

// Global-memory layout: threads (workspace slots) of a launch over `total` cells, at most
// what fits in kGlobalWorkBytes of workspace.
constexpr size_t kGlobalWorkBytes = size_t(16) << 30;

static long long global_slots(const Mech &m, long long total)
{
    // one wavefront per slot; more slots than wavefronts resident on the device only queue
    const size_t per = sizeof(double) * global_work_doubles_per_slot(m.h.ns, m.tab.ntb);
    long long cap = std::min<long long>((long long)(kGlobalWorkBytes / per), 16384);
    if (cap < 1) cap = 1;
    return std::min(std::max(total, 1LL), cap);
}

static size_t global_work_doubles(const Mech &m, long long total)
{
    return global_work_doubles_per_slot(m.h.ns, m.tab.ntb) * (size_t)global_slots(m, total);
}

// Launch one kernel over the spans in a (all of mechanism m) on stream st.  The work counter
// a.counter must already be zero (stream order).  gwork: the workspace of a global-layout
// launch (global_work_doubles doubles); NULL allocates it stream-ordered on st.
static kin_status launch_spans(kin_ctx *ctx, Mech &m, AdvanceArgs &a, kin_precision prec, int layout,
                               int block, hipStream_t st, double *gwork = nullptr, long long gslots = 0)
{
    const bool f32 = prec == KIN_FP32_LU;
    a.ns = m.h.ns;
    if (layout == KIN_LAYOUT_LANE) {
        if (m.h.ns > kLaneNsMax) return err(KIN_EINVAL, "lane layout needs ns <= 15");
        // a launch with a schedule trace runs the recorder build of the same kernels
        kin_status s = a.trace ? build_lane_trace(ctx, m, block) : build_lane(ctx, m, block);
        if (s != KIN_OK) return s;
        hipFunction_t fn = a.trace ? (f32 ? m.lane_f32_tr : m.lane_f64_tr) : (f32 ? m.lane_f32 : m.lane_f64);
        int per_cu = 0;
        KIN_HIP(ctx, hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, 0));
        if (per_cu < 1) per_cu = 1;
        // persistent lanes: one resident wave set; more blocks than fit would only wait
        const long long grid = std::min<long long>((a.total + block - 1) / block, (long long)per_cu * ctx->num_cu);
        a.K = m.kconst;
        void *params[] = {&a};
        KIN_HIP(ctx, hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, block, 1, 1, 0, st, params, nullptr));
    } else if (layout == KIN_LAYOUT_GLOBAL) {
        const long long S = gslots > 0 ? std::min(gslots, global_slots(m, a.total)) : global_slots(m, a.total);
        if (gwork) {
            KIN_HIP(ctx, launch_global(m.tab, a, f32, gwork, S, st));
        } else {
            double *w = nullptr;
            KIN_HIP(ctx, hipMallocAsync(reinterpret_cast<void **>(&w), sizeof(double) * global_work_doubles(m, a.total), st));
            KIN_HIP(ctx, launch_global(m.tab, a, f32, w, S, st));
            KIN_HIP(ctx, hipFreeAsync(w, st));
        }
    } else {
        if (m.h.ns > kWaveNsMax) return err(KIN_EINVAL, "wave layout needs ns <= 63");
        const long long blocks = (a.total + block - 1) / block;
        if (blocks > 0x7fffffffLL) return err(KIN_EINVAL, "too many cells for one wave-layout launch");
        KIN_HIP(ctx, launch_wave(m.tab, a, f32, block, (int)blocks, st));
    }
    return KIN_OK;
}

static bool opts_ok(const kin_solver_opts &o)
{
    return o.rtol >= 0 && o.atol_Y >= 0 && o.atol_T >= 0 && o.y_neg >= 0 && o.k_max >= 1 && o.L_max >= 0 &&
           o.L_max <= 62 && o.L_forced <= 30 && o.L_forced >= -1 && o.max_iters >= 1 &&
           o.layout >= KIN_LAYOUT_AUTO && o.layout <= KIN_LAYOUT_GLOBAL && o.diverge_ratio >= 0;
}

// One kernel launch of a multi-instance advance: instances of one mechanism and layout, at most
// kMaxSpans of them.
struct Launch {
    Mech *m;
    int layout, block;
    AdvanceArgs a;
};

// Group instances by (mechanism, layout), at most kMaxSpans per launch, in a fixed order.
static void plan_launches(kin_ctx *ctx, const int32_t *ids, const double *dts, int n, const kin_solver_opts &o,
                          int prec, std::vector<Launch> &launches)
{
    std::map<int, std::vector<int>> groups;  // mechanism -> positions
    std::map<int, long long> cells;          // mechanism -> cells over its instances
    for (int k = 0; k < n; ++k) {
        Inst &in = *ctx->insts[ids[k]];
        groups[in.mech].push_back(k);
        cells[in.mech] += in.n;
    }
    for (auto &g : groups) {
        Mech &m = *ctx->mechs[g.first];
        int layout, block;
        layout_of(m, o, prec, cells[g.first], layout, block);
        for (size_t off = 0; off < g.second.size(); off += kMaxSpans) {
            Launch L;
            L.m = &m; L.layout = layout; L.block = block;
            std::memset(&L.a, 0, sizeof L.a);
            fill_opts(L.a, o);
            long long total = 0;
            const size_t cnt = std::min<size_t>(kMaxSpans, g.second.size() - off);
            for (size_t q = 0; q < cnt; ++q) {
                const int k = g.second[off + q];
                Inst &in = *ctx->insts[ids[k]];
                L.a.span[q].start = total;
                L.a.span[q].n = in.n;
                L.a.span[q].dt = dts[k];
                L.a.span[q].base = static_cast<char *>(in.buf);
                total += in.n;
            }
            L.a.nspan = (int)cnt;
            L.a.total = total;
            launches.push_back(L);
        }
    }
}

// Batched advance: instances grouped by (mechanism, layout), at most kMaxSpans per launch, each
// launch preceded by a kernel that zeroes its work counter, launches of different groups on
// parallel branches; captured once into a graph and replayed while the description is unchanged.
static kin_status advance_batch(kin_ctx *ctx, const int32_t *ids, const double *dts, int n, kin_precision prec,
                                const kin_solver_opts &o, hipStream_t user)
{
    std::vector<Launch> launches;
    plan_launches(ctx, ids, dts, n, o, prec, launches);
    const int nl = (int)launches.size();
    // key: everything the captured kernels depend on
    std::string key(reinterpret_cast<const char *>(&prec), sizeof prec);
    key.append(reinterpret_cast<const char *>(&o), sizeof o);
    for (const Launch &L : launches) {
        key.append(reinterpret_cast<const char *>(&L.layout), sizeof(int));
        key.append(reinterpret_cast<const char *>(&L.block), sizeof(int));
        key.append(reinterpret_cast<const char *>(&L.m), sizeof(void *));
        key.append(reinterpret_cast<const char *>(L.a.span), sizeof(CellSpan) * L.a.nspan);
    }
    auto pit = ctx->plans.find(key);
    if (pit == ctx->plans.end()) {
        if (ctx->ncounters < nl) {
            // existing graphs point at the old counters
            for (auto &kv : ctx->plans) {
                KIN_HIP(ctx, hipGraphExecDestroy(kv.second.exec));
                if (kv.second.gwork) KIN_HIP(ctx, hipFree(kv.second.gwork));
            }
            ctx->plans.clear();
            if (ctx->counters) KIN_HIP(ctx, hipFree(ctx->counters));
            ctx->ncounters = std::max(nl, 16);
            KIN_HIP(ctx, hipMalloc(&ctx->counters, sizeof(unsigned long long) * ctx->ncounters));
        }
        while ((int)ctx->cap.size() < nl) {
            hipStream_t sx;
            KIN_HIP(ctx, hipStreamCreateWithFlags(&sx, hipStreamNonBlocking));
            ctx->cap.push_back(sx);
            hipEvent_t ev;
            KIN_HIP(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            ctx->join.push_back(ev);
        }
        if (!ctx->fork) KIN_HIP(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
        // compile lane modules and allocate the global layout's workspace outside the capture
        std::vector<size_t> goff(nl, 0);
        size_t gtotal = 0;
        for (int q = 0; q < nl; ++q) {
            Launch &L = launches[q];
            if (L.layout == KIN_LAYOUT_LANE) {
                kin_status s = build_lane(ctx, *L.m, L.block);
                if (s != KIN_OK) return s;
            } else if (L.layout == KIN_LAYOUT_GLOBAL) {
                goff[q] = gtotal;
                gtotal += global_work_doubles(*L.m, L.a.total);
            }
        }
        double *gw = nullptr;
        if (gtotal) KIN_HIP(ctx, hipMalloc(reinterpret_cast<void **>(&gw), sizeof(double) * gtotal));
        hipStream_t c0 = ctx->cap[0];
        KIN_HIP(ctx, hipStreamBeginCapture(c0, hipStreamCaptureModeThreadLocal));
        kin_status cs = KIN_OK;
        hipError_t he = hipEventRecord(ctx->fork, c0);
        for (int q = 0; q < nl && he == hipSuccess && cs == KIN_OK; ++q) {
            hipStream_t sq = ctx->cap[q];
            if (q > 0) he = hipStreamWaitEvent(sq, ctx->fork, 0);
            if (he != hipSuccess) break;
            launches[q].a.counter = ctx->counters + q;
            he = launch_zero_u64(ctx->counters + q, 1, sq);
            if (he != hipSuccess) break;
            cs = launch_spans(ctx, *launches[q].m, launches[q].a, prec, launches[q].layout, launches[q].block, sq,
                              launches[q].layout == KIN_LAYOUT_GLOBAL ? gw + goff[q] : nullptr);
            if (cs == KIN_OK && q > 0) {
                he = hipEventRecord(ctx->join[q], sq);
                if (he == hipSuccess) he = hipStreamWaitEvent(c0, ctx->join[q], 0);
            }
        }
        hipGraph_t graph = nullptr;
        hipError_t he2 = hipStreamEndCapture(c0, &graph);
        if (cs != KIN_OK) {
            if (graph) hipGraphDestroy(graph);
            if (gw) hipFree(gw);
            return cs;
        }
        if (he != hipSuccess || he2 != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            if (gw) hipFree(gw);
            ctx->poisoned = true;
            return err(KIN_EDEVICE, std::string("graph capture: ") + hipGetErrorString(he != hipSuccess ? he : he2));
        }
        Plan plan;
        plan.gwork = gw;
        hipError_t he3 = hipGraphInstantiate(&plan.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (he3 != hipSuccess) {
            if (gw) hipFree(gw);
            ctx->poisoned = true;
            return err(KIN_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(he3));
        }
        plan.insts.assign(ids, ids + n);
        pit = ctx->plans.emplace(key, plan).first;
    }
    KIN_HIP(ctx, hipGraphLaunch(pit->second.exec, user));
    return KIN_OK;
}

// Arguments of an advance (either entry point); ctx->mu must be held for the instance checks.
static kin_status check_advance(kin_ctx *ctx, const int32_t *inst_ids, const double *dts, int32_t n,
                                kin_precision prec, const kin_solver_opts *sopt, kin_solver_opts &o)
{
    if (n < 1 || !inst_ids || !dts) return err(KIN_EINVAL, "bad instance list");
    if (prec != KIN_FP64 && prec != KIN_FP32_LU) return err(KIN_EINVAL, "bad precision");
    kin_default_solver_opts(&o);
    if (sopt) o = *sopt;
    if (!opts_ok(o)) return err(KIN_EINVAL, "bad solver options");
    if (o.point_implicit && prec != KIN_FP64)
        return err(KIN_EINVAL, "the point-implicit step has no Newton refinement and runs in FP64 only");
    for (int k = 0; k < n; ++k) {
        auto it = ctx->insts.find(inst_ids[k]);
        if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
        if (!std::isfinite(dts[k]) || dts[k] < 0) return err(KIN_EINVAL, "dt must be finite and >= 0");
        for (int q = 0; q < k; ++q)
            if (inst_ids[q] == inst_ids[k]) return err(KIN_EINVAL, "an instance appears twice in one advance");
    }
    return KIN_OK;
}

kin_status kin_advance(kin_ctx *ctx, const int32_t *inst_ids, const double *dts, int32_t n,
                       kin_precision prec, const kin_solver_opts *sopt, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    kin_solver_opts o;
    if ((s = check_advance(ctx, inst_ids, dts, n, prec, sopt, o)) != KIN_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n > 1) {
        s = advance_batch(ctx, inst_ids, dts, n, prec, o, st);
        if (s == KIN_OK)
            for (int k = 0; k < n; ++k) ctx->insts[inst_ids[k]]->iters_current = true;
        return s;
    }
    Inst &in = *ctx->insts[inst_ids[0]];
    Mech &m = *ctx->mechs[in.mech];
    int layout, block;
    layout_of(m, o, prec, in.n, layout, block);
    AdvanceArgs a;
    std::memset(&a, 0, sizeof a);
    fill_opts(a, o);
    a.span[0].start = 0;
    a.span[0].n = in.n;
    a.span[0].dt = dts[0];
    a.span[0].base = static_cast<char *>(in.buf);
    a.nspan = 1;
    a.total = in.n;
    a.counter = in.counter;
    // cost order: cells that needed many iterations in the previous advance are taken first;
    // in the lane layout a first advance orders by the source term's temperature change.  The
    // order's scan also clears the work counter; without an order a kernel of its own does
    const long long order_min = layout == KIN_LAYOUT_LANE ? kOrderMinLaneCells : kOrderMinCells;
    if (!o.point_implicit && in.n >= order_min && in.n <= 0x7fffffffLL) {
        const Arena ar = arena_at(static_cast<char *>(in.buf), in.n, m.h.ns);
        if (in.iters_current) {
            KIN_HIP(ctx, launch_cost_order(in.iters, in.n, false, ar.order, ar.ocount, in.counter, st));
            a.span[0].order = ar.order;
        } else if (layout == KIN_LAYOUT_LANE && m.h.ns <= kLaneNsMax) {
            if ((s = build_lane(ctx, m, block)) != KIN_OK) return s;
            a.K = m.kconst;
            int *key = ar.okey;
            void *params[] = {&a, &key};
            const long long grid = (in.n + block - 1) / block;
            KIN_HIP(ctx, hipModuleLaunchKernel(m.lane_cost, (unsigned)grid, 1, 1, block, 1, 1, 0, st, params, nullptr));
            KIN_HIP(ctx, launch_cost_order(ar.okey, in.n, true, ar.order, ar.ocount, in.counter, st));
            a.span[0].order = ar.order;
        }
    }
    if (!a.span[0].order) KIN_HIP(ctx, launch_zero_u64(in.counter, 1, st));
    hipEvent_t k1 = nullptr;
    if (ctx->time_kernels) {
        if (ctx->kev_used == ctx->kev.size()) {
            hipEvent_t a0, a1;
            KIN_HIP(ctx, hipEventCreate(&a0));
            KIN_HIP(ctx, hipEventCreate(&a1));
            ctx->kev.push_back({a0, a1});
        }
        KIN_HIP(ctx, hipEventRecord(ctx->kev[ctx->kev_used].first, st));
        k1 = ctx->kev[ctx->kev_used].second;
    }
    s = launch_spans(ctx, m, a, prec, layout, block, st);
    if (s != KIN_OK) return s;
    if (k1) {
        KIN_HIP(ctx, hipEventRecord(k1, st));
        ctx->kev_used++;
    }
    in.iters_current = true;
    return KIN_OK;
}

kin_status kin_kernel_times(kin_ctx *ctx, double *ms, int32_t cap, int32_t *count)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!count || cap < 0 || (cap > 0 && !ms)) return err(KIN_EINVAL, "bad kernel-time arguments");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    *count = (int32_t)ctx->kev_used;
    for (size_t k = 0; k < ctx->kev_used; ++k) {
        KIN_HIP(ctx, hipEventSynchronize(ctx->kev[k].second));
        if ((int32_t)k < cap) {
            float t = 0.f;
            KIN_HIP(ctx, hipEventElapsedTime(&t, ctx->kev[k].first, ctx->kev[k].second));
            ms[k] = t;
        }
    }
    ctx->kev_used = 0;
    return KIN_OK;
}

kin_status kin_advance_trace(kin_ctx *ctx, int32_t inst_id, double dt, kin_precision prec,
                             const kin_solver_opts *sopt, int32_t words, uint64_t *trace, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    kin_solver_opts o;
    if ((s = check_advance(ctx, &inst_id, &dt, 1, prec, sopt, o)) != KIN_OK) return s;
    if (!trace || words < 2 || words > 4096) return err(KIN_EINVAL, "trace needs a buffer of 2..4096 words per cell");
    Inst &in = *ctx->insts[inst_id];
    Mech &m = *ctx->mechs[in.mech];
    int layout, block;
    layout_of(m, o, prec, in.n, layout, block);
    AdvanceArgs a;
    std::memset(&a, 0, sizeof a);
    fill_opts(a, o);
    a.span[0].n = in.n;
    a.span[0].dt = dt;
    a.span[0].base = static_cast<char *>(in.buf);
    a.nspan = 1;
    a.total = in.n;
    a.counter = in.counter;
    a.trace = reinterpret_cast<unsigned long long *>(trace);
    a.trace_words = words;
    hipStream_t st = static_cast<hipStream_t>(stream);
    KIN_HIP(ctx, launch_zero_u64(in.counter, 1, st));
    s = launch_spans(ctx, m, a, prec, layout, block, st);
    if (s == KIN_OK) in.iters_current = true;
    return s;
}

kin_status kin_advance_noalloc(kin_ctx *ctx, const int32_t *inst_ids, const double *dts, int32_t n,
                               kin_precision prec, const kin_solver_opts *sopt, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    kin_solver_opts o;
    if ((s = check_advance(ctx, inst_ids, dts, n, prec, sopt, o)) != KIN_OK) return s;
    if (n > kScratchLaunches)
        return err(KIN_EINVAL, "kin_advance_noalloc takes at most " + std::to_string(kScratchLaunches) +
                                   " instances per call (one fixed work counter per launch)");
    if (!ctx->scratch) return err(KIN_EDEVICE, "no fixed device memory on this device");
    std::vector<Launch> launches;
    plan_launches(ctx, inst_ids, dts, n, o, prec, launches);
    if ((int)launches.size() > kScratchLaunches) return err(KIN_EINVAL, "too many launches for the fixed counters");
    unsigned long long *counters = reinterpret_cast<unsigned long long *>(ctx->scratch);
    double *work = reinterpret_cast<double *>(ctx->scratch + kScratchWorkOffset);
    const size_t work_bytes = kScratchBytes - kScratchWorkOffset;
    // everything that would allocate (lane kernels not compiled for this block) is refused up
    // front, before any launch
    for (const Launch &L : launches) {
        if (L.layout == KIN_LAYOUT_LANE && !(L.m->mod && L.m->lane_block == L.block))
            return err(KIN_EINVAL, "the lane-layout kernels of this mechanism are not compiled for " +
                                       std::to_string(L.block) + " threads per block; kin_set_layout or kin_advance compiles them");
        if (L.layout == KIN_LAYOUT_GLOBAL &&
            sizeof(double) * global_work_doubles_per_slot(L.m->h.ns, L.m->tab.ntb) > work_bytes)
            return err(KIN_EINVAL, "one cell's matrix exceeds the fixed workspace");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (size_t q = 0; q < launches.size(); ++q) {
        Launch &L = launches[q];
        L.a.counter = counters + q;
        KIN_HIP(ctx, launch_zero_u64(counters + q, 1, st));
        long long gslots = 0;
        if (L.layout == KIN_LAYOUT_GLOBAL)  // launches are stream-ordered, so they share it
            gslots = (long long)(work_bytes / (sizeof(double) * global_work_doubles_per_slot(L.m->h.ns, L.m->tab.ntb)));
        s = launch_spans(ctx, *L.m, L.a, prec, L.layout, L.block, st, L.layout == KIN_LAYOUT_GLOBAL ? work : nullptr, gslots);
        if (s != KIN_OK) return s;
    }
    for (int k = 0; k < n; ++k) ctx->insts[inst_ids[k]]->iters_current = true;
    return KIN_OK;
}

kin_status kin_download(kin_ctx *ctx, int32_t inst_id, double *T, double *Y, double *e0,
                        int32_t *status, int32_t *level, int32_t *iters, kin_mem where,
                        void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->insts.find(inst_id);
    if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
    const Inst &in = *it->second;
    const int ns = ctx->mechs[in.mech]->h.ns;
    if (!mem_ok(where)) return err(KIN_EINVAL, "bad memory kind");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const hipMemcpyKind kind = out_kind(where);
    const size_t nd = sizeof(double) * (size_t)in.n, ni = sizeof(int) * (size_t)in.n;
    if (T) KIN_HIP(ctx, hipMemcpyAsync(T, in.T, nd, kind, st));
    if (Y) KIN_HIP(ctx, hipMemcpyAsync(Y, in.Y, nd * ns, kind, st));
    if (e0) KIN_HIP(ctx, hipMemcpyAsync(e0, in.e0, nd, kind, st));
    if (status) KIN_HIP(ctx, hipMemcpyAsync(status, in.status, ni, kind, st));
    if (level) KIN_HIP(ctx, hipMemcpyAsync(level, in.level, ni, kind, st));
    if (iters) KIN_HIP(ctx, hipMemcpyAsync(iters, in.iters, ni, kind, st));
    if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipStreamSynchronize(st));
    return KIN_OK;
}

kin_status kin_download_schedule(kin_ctx *ctx, int32_t inst_id, uint64_t *sched, kin_mem where,
                                 void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!sched) return err(KIN_EINVAL, "NULL destination");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->insts.find(inst_id);
    if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
    const Inst &in = *it->second;
    if (!mem_ok(where)) return err(KIN_EINVAL, "bad memory kind");
    hipStream_t st = static_cast<hipStream_t>(stream);
    KIN_HIP(ctx, hipMemcpyAsync(sched, in.sched, sizeof(uint64_t) * (size_t)in.n, out_kind(where), st));
    if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipStreamSynchronize(st));
    return KIN_OK;
}

kin_status kin_sync(kin_ctx *ctx, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    KIN_HIP(ctx, hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    return KIN_OK;
}

kin_status kin_stream_create(kin_ctx *ctx, int32_t cu_begin, int32_t cu_end, void **stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!stream || cu_begin < 0 || cu_end > ctx->num_cu || cu_begin >= cu_end)
        return err(KIN_EINVAL, "need 0 <= cu_begin < cu_end <= number of compute units");
    std::vector<uint32_t> mask((ctx->num_cu + 31) / 32, 0u);
    for (int c = cu_begin; c < cu_end; ++c) mask[c / 32] |= 1u << (c % 32);
    hipStream_t st = nullptr;
    KIN_HIP(ctx, hipExtStreamCreateWithCUMask(&st, (uint32_t)mask.size(), mask.data()));
    *stream = st;
    return KIN_OK;
}

kin_status kin_stream_destroy(kin_ctx *ctx, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!stream) return err(KIN_EINVAL, "NULL stream");
    KIN_HIP(ctx, hipStreamDestroy(static_cast<hipStream_t>(stream)));
    return KIN_OK;
}

kin_status kin_instance_release(kin_ctx *ctx, int32_t inst_id)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->insts.find(inst_id);
    if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
    for (auto pit = ctx->plans.begin(); pit != ctx->plans.end();) {
        if (std::find(pit->second.insts.begin(), pit->second.insts.end(), inst_id) != pit->second.insts.end()) {
            KIN_HIP(ctx, hipGraphExecDestroy(pit->second.exec));
            if (pit->second.gwork) KIN_HIP(ctx, hipFree(pit->second.gwork));
            pit = ctx->plans.erase(pit);
        } else {
            ++pit;
        }
    }
    if (ctx->pool) pool_free(ctx, it->second->buf, it->second->bytes);
    else KIN_HIP(ctx, hipFree(it->second->buf));
    ctx->in_use -= it->second->bytes;
    ctx->mechs[it->second->mech]->refs--;
    ctx->insts.erase(it);
    return KIN_OK;
}

kin_status kin_footprint(const kin_ctx *ctx, int32_t mech_id, int64_t n_cells, kin_precision,
                         uint64_t *bytes)
{
    if (!ctx || !bytes || n_cells < 0) return err(KIN_EINVAL, "bad footprint arguments");
    auto it = ctx->mechs.find(mech_id);
    if (it == ctx->mechs.end()) return err(KIN_ENOTFOUND, "unknown mechanism id");
    *bytes = inst_bytes(it->second->h.ns, n_cells);
    return KIN_OK;
}

kin_status kin_query(const kin_ctx *ctx, int32_t what, int64_t arg, void *out)
{
    if (!ctx || !out) return err(KIN_EINVAL, "bad query arguments");
    switch (what) {
    case KIN_Q_BYTES_IN_USE:
        *static_cast<uint64_t *>(out) = ctx->in_use;
        return KIN_OK;
    case KIN_Q_NUM_CU:
        *static_cast<int32_t *>(out) = ctx->num_cu;
        return KIN_OK;
    case KIN_Q_LARGEST_FREE:
        *static_cast<uint64_t *>(out) = ctx->pool ? pool_largest(ctx) : 0;
        return KIN_OK;
    case KIN_Q_LAYOUT:
    case KIN_Q_BLOCK:
    case KIN_Q_JIT_SECONDS: {
        auto it = ctx->mechs.find((int)arg);
        if (it == ctx->mechs.end()) return err(KIN_ENOTFOUND, "unknown mechanism id");
        if (what == KIN_Q_LAYOUT) *static_cast<int32_t *>(out) = it->second->layout;
        else if (what == KIN_Q_BLOCK) *static_cast<int32_t *>(out) = it->second->block;
        else *static_cast<double *>(out) = it->second->jit_seconds;
        return KIN_OK;
    }
    case KIN_Q_TUNED: {
        auto it = ctx->mechs.find((int)arg);
        if (it == ctx->mechs.end()) return err(KIN_ENOTFOUND, "unknown mechanism id");
        int32_t *p = static_cast<int32_t *>(out);
        for (int prec = 0; prec < 2; ++prec)
            for (int c = 0; c < 5; ++c) {
                auto t = it->second->tuned.find({prec, c});
                p[2 * (5 * prec + c)] = t == it->second->tuned.end() ? -1 : t->second.first;
                p[2 * (5 * prec + c) + 1] = t == it->second->tuned.end() ? -1 : t->second.second;
            }
        return KIN_OK;
    }
    case KIN_Q_DEVICE_PTRS: {
        auto it = ctx->insts.find((int)arg);
        if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
        const Inst &in = *it->second;
        uint64_t *p = static_cast<uint64_t *>(out);
        p[0] = (uint64_t)(uintptr_t)in.rho; p[1] = (uint64_t)(uintptr_t)in.e0;
        p[2] = (uint64_t)(uintptr_t)in.T; p[3] = (uint64_t)(uintptr_t)in.Y;
        p[4] = (uint64_t)(uintptr_t)in.status; p[5] = (uint64_t)(uintptr_t)in.level;
        p[6] = (uint64_t)(uintptr_t)in.iters;
        return KIN_OK;
    }
    default:
        return err(KIN_EINVAL, "unknown query");
    }
}

kin_status kin_autotune(kin_ctx *ctx, int32_t mech_id, int32_t inst_id, double dt, kin_precision prec,
                        int32_t *layout_out, int32_t *block_out, double *best_ms)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!std::isfinite(dt) || dt < 0) return err(KIN_EINVAL, "dt must be finite and >= 0");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto mit = ctx->mechs.find(mech_id);
    auto iit = ctx->insts.find(inst_id);
    if (mit == ctx->mechs.end() || iit == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown id");
    Mech &m = *mit->second;
    Inst &in = *iit->second;
    if (in.mech != mech_id) return err(KIN_EINVAL, "instance belongs to another mechanism");
    std::vector<std::pair<int, int>> cand;
    if (m.h.ns <= kLaneNsMax)
        for (int b : {64, 128, 256})
            if (lane_block_ok(m.h.ns, b)) cand.push_back({KIN_LAYOUT_LANE, b});
    if (m.h.ns <= kWaveNsMax) {
        for (int b : {1, 2, 4})
            if (wave_lds_bytes(m.tab, false) * (size_t)b <= 65536) cand.push_back({KIN_LAYOUT_WAVE, b});
    } else {
        cand.push_back({KIN_LAYOUT_GLOBAL, 64});
    }
    void *save = nullptr;
    const bool iters_was_current = in.iters_current;  // the saved arena's counts, restored with it
    KIN_HIP(ctx, hipMalloc(&save, in.bytes));
    KIN_HIP(ctx, hipMemcpy(save, in.buf, in.bytes, hipMemcpyDeviceToDevice));
    hipEvent_t e0, e1;
    KIN_HIP(ctx, hipEventCreate(&e0));
    KIN_HIP(ctx, hipEventCreate(&e1));
    const int old_layout = m.layout, old_block = m.block;
    const auto old_tuned = m.tuned;
    double best = 1e300;
    std::pair<int, int> win = {old_layout, old_block};
    kin_solver_opts o;
    kin_default_solver_opts(&o);
    for (const auto &c : cand) {
        if ((s = kin_set_layout(ctx, mech_id, c.first, c.second)) != KIN_OK) break;
        KIN_HIP(ctx, hipMemcpy(in.buf, save, in.bytes, hipMemcpyDeviceToDevice));
        // one untimed launch loads the module and warms the caches; candidates are timed in
        // index order
        in.iters_current = false;
        if ((s = kin_advance(ctx, &inst_id, &dt, 1, prec, &o, nullptr)) != KIN_OK) break;
        KIN_HIP(ctx, hipMemcpy(in.buf, save, in.bytes, hipMemcpyDeviceToDevice));
        in.iters_current = false;
        KIN_HIP(ctx, hipEventRecord(e0, nullptr));
        if ((s = kin_advance(ctx, &inst_id, &dt, 1, prec, &o, nullptr)) != KIN_OK) break;
        KIN_HIP(ctx, hipEventRecord(e1, nullptr));
        KIN_HIP(ctx, hipEventSynchronize(e1));
        float ms = 0.f;
        KIN_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) { best = ms; win = c; }
    }
    hipMemcpy(in.buf, save, in.bytes, hipMemcpyDeviceToDevice);
    in.iters_current = iters_was_current;
    hipFree(save);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    // the mechanism keeps its default layout; the choice applies to launches of this size class
    kin_set_layout(ctx, mech_id, old_layout, old_block);
    m.tuned = old_tuned;
    if (s != KIN_OK) return s;
    const int cls = size_class(in.n);
    m.tuned[{(int)prec, cls}] = win;
    auto cache = tune_read(ctx->tune_cache);
    cache[tune_key(ctx, m, prec) + "-c" + std::to_string(cls)] = {(double)win.first, (double)win.second, best};
    tune_write(ctx->tune_cache, cache);
    if (layout_out) *layout_out = win.first;
    if (block_out) *block_out = win.second;
    if (best_ms) *best_ms = best;
    return KIN_OK;
}

kin_status kin_fluid_create(kin_ctx *ctx, int32_t mech_id, int32_t nx, int32_t ny, double dx, double dy,
                            int32_t bc, int32_t *fluid_id)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!fluid_id || nx < 1 || ny < 1 || !(dx > 0.0) || !(dy > 0.0) || !std::isfinite(dx) || !std::isfinite(dy) ||
        (bc != KIN_BC_PERIODIC && bc != KIN_BC_OUTFLOW))
        return err(KIN_EINVAL, "bad fluid grid arguments");
    if ((long long)nx * ny > (1LL << 31)) return err(KIN_EINVAL, "fluid grid too large");
    // the six-cell stencil wraps at most once around a periodic direction of three or more cells
    if (bc == KIN_BC_PERIODIC && (nx < 3 || ny < 3))
        return err(KIN_EINVAL, "a periodic fluid grid needs at least 3 cells in each direction");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->mechs.find(mech_id);
    if (it == ctx->mechs.end()) return err(KIN_ENOTFOUND, "unknown mechanism id");
    Mech &m = *it->second;
    std::unique_ptr<Fluid> f(new Fluid());
    f->mech = mech_id;
    f->g = FluidGrid{nx, ny, bc};
    f->dx = dx;
    f->dy = dy;
    // arrays [var][n] with stride n = nx ny (the instance arena's layout of Y), each array
    // starting on a 256-byte boundary
    const size_t n = (size_t)nx * ny, nv = (size_t)m.h.ns + 3;
    const size_t nf = nv * (size_t)(nx + 1) * (ny + 1);
    auto up = [](size_t d) { return (d + 31) & ~(size_t)31; };
    const size_t doubles = 3 * up(nv * n) + 3 * up(n) + 32 + up(nf);
    KIN_HIP(ctx, hipMalloc(&f->buf, sizeof(double) * doubles));
    double *p = static_cast<double *>(f->buf);
    f->Q = p; p += up(nv * n);
    f->Q1 = p; p += up(nv * n);
    f->W = p; p += up(nv * n);
    f->T = p; p += up(n);
    f->KE = p; p += up(n);
    f->Es = p; p += up(n);
    f->speed = reinterpret_cast<unsigned long long *>(p); p += 32;
    f->F = p;
    // Newton start temperature of the first sweep
    std::vector<double> T0(n, 1000.0);
    KIN_HIP(ctx, hipMemcpy(f->T, T0.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    m.refs++;
    const int id = ctx->next_fluid++;
    ctx->fluids[id] = std::move(f);
    *fluid_id = id;
    return KIN_OK;
}

kin_status kin_fluid_release(kin_ctx *ctx, int32_t fluid_id)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->fluids.find(fluid_id);
    if (it == ctx->fluids.end()) return err(KIN_ENOTFOUND, "unknown fluid id");
    ctx->mechs[it->second->mech]->refs--;
    KIN_HIP(ctx, hipFree(it->second->buf));
    ctx->fluids.erase(it);
    return KIN_OK;
}

static kin_status find_fluid(kin_ctx *ctx, int32_t fluid_id, Fluid *&f, Mech *&m)
{
    auto it = ctx->fluids.find(fluid_id);
    if (it == ctx->fluids.end()) return err(KIN_ENOTFOUND, "unknown fluid id");
    f = it->second.get();
    m = ctx->mechs[f->mech].get();
    return KIN_OK;
}

kin_status kin_fluid_upload(kin_ctx *ctx, int32_t fluid_id, const double *Q, kin_mem where, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!Q || !mem_ok(where)) return err(KIN_EINVAL, "bad fluid upload arguments");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Fluid *f;
    Mech *m;
    if ((s = find_fluid(ctx, fluid_id, f, m)) != KIN_OK) return s;
    const size_t bytes = sizeof(double) * ((size_t)m->h.ns + 3) * (size_t)f->g.nx * f->g.ny;
    return copy_in(ctx, f->Q, Q, bytes, where, static_cast<hipStream_t>(stream));
}

kin_status kin_fluid_download(kin_ctx *ctx, int32_t fluid_id, double *Q, kin_mem where, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!Q || !mem_ok(where)) return err(KIN_EINVAL, "bad fluid download arguments");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Fluid *f;
    Mech *m;
    if ((s = find_fluid(ctx, fluid_id, f, m)) != KIN_OK) return s;
    const size_t bytes = sizeof(double) * ((size_t)m->h.ns + 3) * (size_t)f->g.nx * f->g.ny;
    hipStream_t st = static_cast<hipStream_t>(stream);
    KIN_HIP(ctx, hipMemcpyAsync(Q, f->Q, bytes, out_kind(where), st));
    if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipStreamSynchronize(st));
    return KIN_OK;
}

kin_status kin_fluid_max_dt(kin_ctx *ctx, int32_t fluid_id, double cfl, double *dt, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!dt || !(cfl > 0.0)) return err(KIN_EINVAL, "bad CFL arguments");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Fluid *f;
    Mech *m;
    if ((s = find_fluid(ctx, fluid_id, f, m)) != KIN_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    KIN_HIP(ctx, launch_zero_u64(f->speed, 1, st));
    KIN_HIP(ctx, launch_fluid_speed(m->tab, f->g, f->Q, f->W, f->T, f->dx, f->dy, f->speed, st));
    unsigned long long bits = 0;
    KIN_HIP(ctx, hipMemcpyAsync(&bits, f->speed, sizeof bits, hipMemcpyDeviceToHost, st));
    KIN_HIP(ctx, hipStreamSynchronize(st));
    double r;
    std::memcpy(&r, &bits, sizeof r);
    *dt = (r > 0.0 && std::isfinite(r)) ? cfl / r : 0.0;
    return KIN_OK;
}

static kin_status fluid_step(kin_ctx *ctx, Fluid &f, Mech &m, double dt, int y_first, hipStream_t st)
{
    for (int k = 0; k < 2; ++k) {
        const int dir = (k == 0) == (y_first == 0) ? 0 : 1;
        KIN_HIP(ctx, launch_fluid_sweep(m.tab, f.g, dir, dt, dir == 0 ? f.dx : f.dy, f.Q, f.Q1, f.W, f.T, f.F, st));
    }
    return KIN_OK;
}

kin_status kin_fluid_step(kin_ctx *ctx, int32_t fluid_id, double dt, int32_t y_first, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!(dt >= 0.0) || !std::isfinite(dt)) return err(KIN_EINVAL, "dt must be finite and >= 0");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Fluid *f;
    Mech *m;
    if ((s = find_fluid(ctx, fluid_id, f, m)) != KIN_OK) return s;
    return fluid_step(ctx, *f, *m, dt, y_first, static_cast<hipStream_t>(stream));
}

kin_status kin_split_step(kin_ctx *ctx, int32_t fluid_id, int32_t inst_id, double dt, int32_t y_first,
                          kin_precision prec, const kin_solver_opts *sopt, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!(dt >= 0.0) || !std::isfinite(dt)) return err(KIN_EINVAL, "dt must be finite and >= 0");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Fluid *f;
    Mech *m;
    if ((s = find_fluid(ctx, fluid_id, f, m)) != KIN_OK) return s;
    auto iit = ctx->insts.find(inst_id);
    if (iit == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
    const long long n = (long long)f->g.nx * f->g.ny;
    if (iit->second->mech != f->mech || iit->second->n != n)
        return err(KIN_EINVAL, "the instance must hold the fluid grid's cells, of the same mechanism");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((s = fluid_step(ctx, *f, *m, dt, y_first, st)) != KIN_OK) return s;
    // the chemistry sub-step on the same cells: partial densities and sensible energy in, the
    // fluid sweep's last temperatures as the inversion's start values, and back
    KIN_HIP(ctx, launch_fluid_kinetic(f->g, m->h.ns, f->Q, f->KE, f->Es, st));
    // Iteration counts of the instance's previous advance (the chemistry of the previous split
    // step, on the same cells) predict this step's costs as they do for a plain second advance,
    // so they survive the reset for the cost order; the order never changes a cell's result.
    const bool counts = iit->second->iters_current;
    if ((s = kin_state_reset_conserved(ctx, inst_id, f->Q, f->Es, f->T, KIN_MEM_DEVICE, stream)) != KIN_OK) return s;
    iit->second->iters_current = counts;
    if ((s = kin_advance(ctx, &inst_id, &dt, 1, prec, sopt, stream)) != KIN_OK) return s;
    if ((s = kin_download_conserved(ctx, inst_id, f->Q, f->Es, KIN_MEM_DEVICE, stream)) != KIN_OK) return s;
    KIN_HIP(ctx, launch_fluid_energy_back(f->g, m->h.ns, f->Q, f->KE, f->Es, st));
    return KIN_OK;
}

kin_status kin_jit_check(const kin_mech_desc *d, char *log, size_t log_len)
{
    MechHost h;
    std::string msg;
    kin_status s = mech_from_desc(d, h, msg);
    if (s == KIN_OK) {
        if (h.ns > kLaneNsMax) {
            s = KIN_EINVAL;
            msg = "lane layout needs ns <= 15";
        } else {
            std::vector<char> code;
            std::vector<double> consts;
            double secs = 0.0;
            const std::string src = lane_source(h, 64, consts);
            s = rtc_compile(src, "kin_lane.hip", code, msg, &secs);
            if (s == KIN_OK) {
                // and the build with the schedule recorder (kin_advance_trace)
                std::vector<char> code_tr;
                double secs_tr = 0.0;
                s = rtc_compile("#define KIN_TRACE 1\n" + src, "kin_lane_trace.hip", code_tr, msg, &secs_tr);
                if (s == KIN_OK)
                    msg = "compiled " + std::to_string(code.size()) + " bytes in " + std::to_string(secs) +
                          " s, with the schedule recorder " + std::to_string(code_tr.size()) + " bytes\n" + msg;
            }
        }
    }
    if (log && log_len) {
        std::strncpy(log, msg.c_str(), log_len - 1);
        log[log_len - 1] = '\0';
    }
    if (s != KIN_OK) set_error(msg);
    return s;
}

}  // extern "C"
