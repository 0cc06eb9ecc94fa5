// kin_runtime.cpp -- the C ABI of libkin: contexts, device-resident mechanisms and cell
// instances, advance launches, downloads.  See include/kin.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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
    hipFunction_t lane_f64 = nullptr, lane_f32 = nullptr;
    double *kconst = nullptr;  // constant table of the lane kernels
    int lane_block = 0;      // block size the module was compiled for
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
};

// Code objects already compiled in this process, keyed by their source.
static std::mutex g_jit_mu;
static std::unordered_map<std::string, std::pair<std::vector<char>, double>> g_jit_cache;

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static uint64_t inst_bytes(int ns, long long n)
{
    const size_t d = align256(sizeof(double) * (size_t)n);
    const size_t i = align256(sizeof(int) * (size_t)n);
    return (uint64_t)(d * (4 + (size_t)ns) + 3 * i + 256);
}

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
    int next_mech = 1, next_inst = 1;
};

using namespace kin;

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
    if (o && o->tune_cache) c->tune_cache = o->tune_cache;
    else if (const char *env = std::getenv("KIN_TUNE_CACHE")) c->tune_cache = env;
    if ((e = hipSetDevice(c->device)) != hipSuccess) return err(KIN_EDEVICE, hipGetErrorString(e));
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, c->device)) != hipSuccess) return err(KIN_EDEVICE, hipGetErrorString(e));
    c->num_cu = prop.multiProcessorCount;
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
        for (auto &kv : ctx->insts) hipFree(kv.second->buf);
        for (auto &kv : ctx->mechs) {
            if (kv.second->mod) hipModuleUnload(kv.second->mod);
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
    m.lane_block = block;
    m.jit_seconds += secs;
    return KIN_OK;
}

// Pack the device tables of the table-driven kernels.
static kin_status upload_tables(kin_ctx *ctx, Mech &m)
{
    const MechHost &h = m.h;
    const int ns = h.ns, nr = h.nr, ntb = h.ntb;
    const int nchunk = (nr + kChunk - 1) / kChunk;
    std::vector<double> rxd((size_t)nr * 4);
    std::vector<RxnRec> rxc(nr);
    for (int r = 0; r < nr; ++r) {
        const Rxn &x = h.rx[r];
        rxd[4 * r + 0] = x.lnA;
        rxd[4 * r + 1] = x.b;
        rxd[4 * r + 2] = x.Ta;
        rxd[4 * r + 3] = (double)x.dnu;
        RxnRec &p = rxc[r];
        std::memset(&p, 0, sizeof p);
        p.rev = (int8_t)x.rev; p.nreac = (int8_t)x.nreac; p.nprod = (int8_t)x.nprod;
        p.npart = (int8_t)x.npart; p.tb = (int16_t)x.tb;
        for (int j = 0; j < 3; ++j) {
            p.reac_sp[j] = (int8_t)(j < x.nreac ? x.reac_sp[j] : 0);
            p.reac_nu[j] = (int8_t)(j < x.nreac ? x.reac_nu[j] : 0);
            p.prod_sp[j] = (int8_t)(j < x.nprod ? x.prod_sp[j] : 0);
            p.prod_nu[j] = (int8_t)(j < x.nprod ? x.prod_nu[j] : 0);
        }
        for (int j = 0; j < 6; ++j) {
            p.part_sp[j] = (int8_t)(j < x.npart ? x.part[j].sp : 0);
            p.part_nu[j] = (int8_t)(j < x.npart ? x.part[j].nu : 0);
        }
    }
    std::vector<double> effT((size_t)std::max(1, ns * ntb), 0.0), effM((size_t)std::max(1, ntb * ns), 0.0);
    for (int r = 0; r < ntb; ++r)
        for (int k = 0; k < ns; ++k) {
            effT[(size_t)k * ntb + r] = h.eff[(size_t)r * ns + k];
            effM[(size_t)r * ns + k] = h.eff[(size_t)r * ns + k] / h.M[k];
        }
    std::vector<int> tb_ptr(nchunk + 1), tb_list;
    for (int cb = 0; cb < nchunk; ++cb) {
        tb_ptr[cb] = (int)tb_list.size();
        for (int r = cb * kChunk; r < std::min(nr, (cb + 1) * kChunk); ++r)
            if (h.rx[r].tb >= 0) tb_list.push_back(r);
    }
    tb_ptr[nchunk] = (int)tb_list.size();
    // per species row and chunk: reactions with nonzero net coefficient, and sparse entries
    std::vector<int> sp_ptr((size_t)ns * (nchunk + 1)), sp_list, ent_ptr((size_t)ns * (nchunk + 1)), ent_list;
    for (int s = 0; s < ns; ++s) {
        for (int cb = 0; cb < nchunk; ++cb) {
            sp_ptr[(size_t)s * (nchunk + 1) + cb] = (int)sp_list.size();
            ent_ptr[(size_t)s * (nchunk + 1) + cb] = (int)ent_list.size();
            for (int r = cb * kChunk; r < std::min(nr, (cb + 1) * kChunk); ++r) {
                const Rxn &x = h.rx[r];
                const int rl = r - cb * kChunk;
                int nu = 0;
                for (int j = 0; j < x.npart; ++j) if (x.part[j].sp == s) nu = x.part[j].nu;
                if (!nu) continue;
                sp_list.push_back(rl * 16 + (nu + 8));
                for (int j = 0; j < x.npart; ++j)
                    ent_list.push_back(rl | (j << 6) | (x.part[j].sp << 9) | ((nu + 8) << 15));
            }
        }
        sp_ptr[(size_t)s * (nchunk + 1) + nchunk] = (int)sp_list.size();
        ent_ptr[(size_t)s * (nchunk + 1) + nchunk] = (int)ent_list.size();
    }
    if (sp_list.empty()) sp_list.push_back(0);
    if (ent_list.empty()) ent_list.push_back(0);
    if (tb_list.empty()) tb_list.push_back(0);
    // one allocation, 256-byte aligned pieces
    struct Piece { const void *src; size_t bytes; size_t off; };
    std::vector<Piece> pc = {
        {h.nasa.data(), sizeof(double) * h.nasa.size(), 0}, {h.Tmid.data(), sizeof(double) * ns, 0},
        {h.M.data(), sizeof(double) * ns, 0}, {rxd.data(), sizeof(double) * rxd.size(), 0},
        {rxc.data(), sizeof(RxnRec) * rxc.size(), 0}, {effT.data(), sizeof(double) * effT.size(), 0},
        {effM.data(), sizeof(double) * effM.size(), 0}, {tb_ptr.data(), sizeof(int) * tb_ptr.size(), 0},
        {tb_list.data(), sizeof(int) * tb_list.size(), 0}, {sp_ptr.data(), sizeof(int) * sp_ptr.size(), 0},
        {sp_list.data(), sizeof(int) * sp_list.size(), 0}, {ent_ptr.data(), sizeof(int) * ent_ptr.size(), 0},
        {ent_list.data(), sizeof(int) * ent_list.size(), 0}};
    size_t total = 0;
    for (Piece &p : pc) { p.off = total; total = align256(total + p.bytes); }
    std::vector<char> host(total, 0);
    for (const Piece &p : pc) std::memcpy(&host[p.off], p.src, p.bytes);
    KIN_HIP(ctx, hipMalloc(&m.dbuf, total));
    m.dbytes = total;
    KIN_HIP(ctx, hipMemcpy(m.dbuf, host.data(), total, hipMemcpyHostToDevice));
    char *b = static_cast<char *>(m.dbuf);
    WaveTables &t = m.tab;
    t.ns = ns; t.nr = nr; t.ntb = ntb; t.nchunk = nchunk;
    t.lnPaR = std::log(kPatmCgs / kRuCgs);
    t.nasa = reinterpret_cast<const double *>(b + pc[0].off);
    t.Tmid = reinterpret_cast<const double *>(b + pc[1].off);
    t.M = reinterpret_cast<const double *>(b + pc[2].off);
    t.rxd = reinterpret_cast<const double *>(b + pc[3].off);
    t.rxc = reinterpret_cast<const RxnRec *>(b + pc[4].off);
    t.effT = reinterpret_cast<const double *>(b + pc[5].off);
    t.effM = reinterpret_cast<const double *>(b + pc[6].off);
    t.tb_ptr = reinterpret_cast<const int *>(b + pc[7].off);
    t.tb_list = reinterpret_cast<const int *>(b + pc[8].off);
    t.sp_ptr = reinterpret_cast<const int *>(b + pc[9].off);
    t.sp_list = reinterpret_cast<const int *>(b + pc[10].off);
    t.ent_ptr = reinterpret_cast<const int *>(b + pc[11].off);
    t.ent_list = reinterpret_cast<const int *>(b + pc[12].off);
    return KIN_OK;
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
    } else {
        m->layout = KIN_LAYOUT_WAVE;
        m->block = 2;
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
        if (block != 64 && block != 128 && block != 256) return err(KIN_EINVAL, "lane block must be 64, 128 or 256");
        if ((s = build_lane(ctx, m, block)) != KIN_OK) return s;
    } else if (layout == KIN_LAYOUT_WAVE) {
        if (block < 1 || block > 4) return err(KIN_EINVAL, "wave layout takes 1..4 wavefronts per block");
    } else {
        return err(KIN_EINVAL, "layout must be LANE or WAVE");
    }
    m.layout = layout;
    m.block = block;
    return KIN_OK;
}

static kin_status copy_in(kin_ctx *ctx, void *dst, const void *src, size_t bytes, kin_mem where,
                          hipStream_t st)
{
    if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    else KIN_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
    return KIN_OK;
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

kin_status kin_state_upload(kin_ctx *ctx, int32_t mech_id, int64_t n_cells, const double *rho,
                            const double *T, const double *Y, const double *e0, kin_mem where,
                            void *stream, int32_t *inst_id)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!inst_id || n_cells < 1 || !rho || !T || !Y) return err(KIN_EINVAL, "bad state arguments");
    if (where != KIN_MEM_HOST && where != KIN_MEM_DEVICE) return err(KIN_EINVAL, "bad memory kind");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->mechs.find(mech_id);
    if (it == ctx->mechs.end()) return err(KIN_ENOTFOUND, "unknown mechanism id");
    Mech &m = *it->second;
    const uint64_t bytes = inst_bytes(m.h.ns, n_cells);
    if (ctx->budget && ctx->in_use + bytes > ctx->budget)
        return err(KIN_ENOMEM, "instance of " + std::to_string(bytes) + " bytes exceeds the context budget");
    std::unique_ptr<Inst> in(new Inst());
    in->mech = mech_id;
    in->n = n_cells;
    in->ld = n_cells;
    in->bytes = bytes;
    KIN_HIP(ctx, hipMalloc(&in->buf, bytes));
    char *b = static_cast<char *>(in->buf);
    const size_t d = align256(sizeof(double) * (size_t)n_cells);
    const size_t i = align256(sizeof(int) * (size_t)n_cells);
    in->rho = reinterpret_cast<double *>(b);
    in->e0 = reinterpret_cast<double *>(b + d);
    in->T = reinterpret_cast<double *>(b + 2 * d);
    in->Y = reinterpret_cast<double *>(b + 3 * d);
    in->sched = reinterpret_cast<unsigned long long *>(b + (3 + (size_t)m.h.ns) * d);
    char *ib = b + (4 + (size_t)m.h.ns) * d;
    in->status = reinterpret_cast<int *>(ib);
    in->level = reinterpret_cast<int *>(ib + i);
    in->iters = reinterpret_cast<int *>(ib + 2 * i);
    in->counter = reinterpret_cast<unsigned long long *>(ib + 3 * i);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((s = fill_state(ctx, *in, m, rho, T, Y, e0, where, st)) != KIN_OK) {
        hipFree(in->buf);
        return s;
    }
    KIN_HIP(ctx, hipMemsetAsync(in->status, 0, 3 * i, st));
    if (where == KIN_MEM_HOST) KIN_HIP(ctx, hipStreamSynchronize(st));
    m.refs++;
    ctx->in_use += bytes;
    const int id = ctx->next_inst++;
    ctx->insts[id] = std::move(in);
    *inst_id = id;
    return KIN_OK;
}

kin_status kin_state_reset(kin_ctx *ctx, int32_t inst_id, const double *rho, const double *T,
                           const double *Y, const double *e0, kin_mem where, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (!rho || !T || !Y) return err(KIN_EINVAL, "NULL state array");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->insts.find(inst_id);
    if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
    Inst &in = *it->second;
    const Mech &m = *ctx->mechs[in.mech];
    return fill_state(ctx, in, m, rho, T, Y, e0, where, static_cast<hipStream_t>(stream));
}

static AdvanceArgs make_args(const Inst &in, double dt, const kin_solver_opts &o)
{
    AdvanceArgs a{};
    a.n = in.n; a.ld = in.ld; a.dt = dt;
    a.rho = in.rho; a.e0 = in.e0; a.T = in.T; a.Y = in.Y;
    a.status = in.status; a.level = in.level; a.iters = in.iters;
    a.rtol = o.rtol; a.atol_Y = o.atol_Y; a.atol_T = o.atol_T; a.y_neg = o.y_neg;
    a.k_max = o.k_max; a.L_max = o.L_max; a.L_forced = o.L_forced; a.max_iters = o.max_iters;
    a.counter = in.counter;
    a.sched = in.sched;
    return a;
}

static kin_status launch_one(kin_ctx *ctx, Mech &m, const Inst &in, double dt, kin_precision prec,
                             const kin_solver_opts &o, hipStream_t st)
{
    int layout = o.layout == KIN_LAYOUT_AUTO ? m.layout : o.layout;
    AdvanceArgs a = make_args(in, dt, o);
    const bool f32 = prec == KIN_FP32_LU;
    KIN_HIP(ctx, hipMemsetAsync(in.counter, 0, sizeof(unsigned long long), st));
    if (layout == KIN_LAYOUT_LANE) {
        if (m.h.ns > kLaneNsMax) return err(KIN_EINVAL, "lane layout needs ns <= 15");
        const int block = (m.layout == KIN_LAYOUT_LANE) ? m.block : 64;
        kin_status s = build_lane(ctx, m, block);
        if (s != KIN_OK) return s;
        hipFunction_t fn = f32 ? m.lane_f32 : m.lane_f64;
        int per_cu = 0;
        KIN_HIP(ctx, hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, 0));
        if (per_cu < 1) per_cu = 1;
        // persistent lanes: one resident wave set; more blocks than fit would only wait
        const long long grid = std::min<long long>((in.n + block - 1) / block, (long long)per_cu * ctx->num_cu);
        a.K = m.kconst;
        void *params[] = {&a};
        KIN_HIP(ctx, hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, block, 1, 1, 0, st, params, nullptr));
    } else {
        const int wpb = (m.layout == KIN_LAYOUT_WAVE) ? m.block : 2;
        const long long blocks = (in.n + wpb - 1) / wpb;
        if (blocks > 0x7fffffffLL) return err(KIN_EINVAL, "too many cells for one wave-layout launch");
        const int grid = (int)blocks;
        KIN_HIP(ctx, launch_wave(m.tab, a, f32, wpb, grid, st));
    }
    return KIN_OK;
}

kin_status kin_advance(kin_ctx *ctx, const int32_t *inst_ids, const double *dts, int32_t n,
                       kin_precision prec, const kin_solver_opts *sopt, void *stream)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    if (n < 1 || !inst_ids || !dts) return err(KIN_EINVAL, "bad instance list");
    if (prec != KIN_FP64 && prec != KIN_FP32_LU) return err(KIN_EINVAL, "bad precision");
    kin_solver_opts o;
    kin_default_solver_opts(&o);
    if (sopt) o = *sopt;
    if (!(o.rtol >= 0) || !(o.atol_Y >= 0) || !(o.atol_T >= 0) || !(o.y_neg >= 0) || o.k_max < 1 ||
        o.L_max < 0 || o.L_max > 62 || o.L_forced > 30 || o.L_forced < -1 || o.max_iters < 1)
        return err(KIN_EINVAL, "bad solver options");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    for (int k = 0; k < n; ++k) {
        auto it = ctx->insts.find(inst_ids[k]);
        if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
        if (!std::isfinite(dts[k]) || dts[k] < 0) return err(KIN_EINVAL, "dt must be finite and >= 0");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int k = 0; k < n; ++k) {
        Inst &in = *ctx->insts[inst_ids[k]];
        Mech &m = *ctx->mechs[in.mech];
        if ((s = launch_one(ctx, m, in, dts[k], prec, o, st)) != KIN_OK) return s;
    }
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
    hipStream_t st = static_cast<hipStream_t>(stream);
    const hipMemcpyKind kind = where == KIN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
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
    hipStream_t st = static_cast<hipStream_t>(stream);
    KIN_HIP(ctx, hipMemcpyAsync(sched, in.sched, sizeof(uint64_t) * (size_t)in.n,
                                where == KIN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
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

kin_status kin_instance_release(kin_ctx *ctx, int32_t inst_id)
{
    kin_status s = enter(ctx);
    if (s != KIN_OK) return s;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->insts.find(inst_id);
    if (it == ctx->insts.end()) return err(KIN_ENOTFOUND, "unknown instance id");
    KIN_HIP(ctx, hipFree(it->second->buf));
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
            s = rtc_compile(lane_source(h, 64, consts), "kin_lane.hip", code, msg, &secs);
            if (s == KIN_OK) msg = "compiled " + std::to_string(code.size()) + " bytes in " + std::to_string(secs) + " s\n" + msg;
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
