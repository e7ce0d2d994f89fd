// capi.hip -- host side of the C ABI declared in include/msmc.h: argument
// validation, field memory, descriptor tables, the sweep / HMC / flow /
// prolongation host loop, HIP graph capture of batched sweeps, the launch-shape
// autotuner and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/msmc.h"
#include "kernels.hpp"

using namespace msmc;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int32_t fail(int32_t code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(SU3_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

// ---------------------------------------------------------------------------
// Small device helpers: tables are written by kernels whose arguments carry
// the values, so updates are ordered on the stream and can be captured.
// ---------------------------------------------------------------------------
namespace {
constexpr int kDescChunk = 20;
struct DescPack {
    LatDesc d[kDescChunk];
    int n, off;
};
constexpr int kIntChunk = 480;
struct IntPack {
    int v[kIntChunk];
    int n, off;
};
}  // namespace

__global__ void k_fill_descs(DescPack p, LatDesc* out)
{
    const int i = threadIdx.x;
    if (i < p.n) out[p.off + i] = p.d[i];
}

__global__ void k_fill_ints(IntPack p, int* out)
{
    for (int i = threadIdx.x; i < p.n; i += blockDim.x) out[p.off + i] = p.v[i];
}

__global__ void k_set_u64(uint64_t* p, uint64_t v)
{
    if (threadIdx.x == 0) *p = v;
}

__global__ void k_zero_u64(unsigned long long* p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

static hipError_t upload_descs(LatDesc* dst, const std::vector<LatDesc>& src, hipStream_t st)
{
    for (size_t o = 0; o < src.size(); o += kDescChunk) {
        DescPack p;
        memset(&p, 0, sizeof p);
        p.n = (int)std::min<size_t>(kDescChunk, src.size() - o);
        p.off = (int)o;
        for (int i = 0; i < p.n; i++) p.d[i] = src[o + i];
        k_fill_descs<<<1, 64, 0, st>>>(p, dst);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static hipError_t upload_ints(int* dst, const std::vector<int>& src, hipStream_t st)
{
    for (size_t o = 0; o < src.size(); o += kIntChunk) {
        IntPack p;
        memset(&p, 0, sizeof p);
        p.n = (int)std::min<size_t>(kIntChunk, src.size() - o);
        p.off = (int)o;
        for (int i = 0; i < p.n; i++) p.v[i] = src[o + i];
        k_fill_ints<<<1, 256, 0, st>>>(p, dst);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Fields
// ---------------------------------------------------------------------------
// Bytes of one slab (one direction and parity) of Vh records of nreal reals
// of rb bytes each: whole tiles of 32 records, rounded up to an odd number
// of 256-byte blocks so that the slabs of one site do not all fall into the
// same cache sets.
static size_t slab_bytes(size_t Vh, int nreal, size_t rb)
{
    const size_t tiles = (Vh + 31) / 32;
    size_t blocks = (tiles * 32 * (size_t)nreal * rb + 255) / 256;
    if (blocks == 0) blocks = 1;
    if ((blocks & 1) == 0) blocks += 1;
    return blocks * 256;
}

struct su3_field_s;

// Launch shape of the phase kernels: block size, XCD remapping and the
// requested site tile (ty, tz, tt; 0 = whole extent, clamped per lattice to
// the largest divisor not above the request).
struct LaunchCfg {
    int block = 256, remap = 1, ty = 0, tz = 0, tt = 1;
    bool operator==(const LaunchCfg& o) const
    {
        return block == o.block && remap == o.remap && ty == o.ty && tz == o.tz && tt == o.tt;
    }
    std::string str() const
    {
        return std::to_string(block) + "," + std::to_string(remap) + "," + std::to_string(ty) + "," +
               std::to_string(tz) + "," + std::to_string(tt);
    }
};

static int largest_divisor_upto(int L, int want)
{
    if (want <= 0 || want >= L) return L;
    for (int t = want; t >= 1; t--)
        if (L % t == 0) return t;
    return 1;
}

// Device tables for a set of lattices of one precision.
struct Plan {
    int nlat = 0;
    int prec = 0;
    LaunchCfg cfg;
    int phase_block = 256, remap = 1;
    LatDesc* d_descs = nullptr;  // nlat entries
    int* d_bbeg_phase = nullptr;
    int* d_bbeg_link = nullptr;
    int* d_bbeg_site = nullptr;
    int* d_bbeg_lw = nullptr;
    int nblk_phase = 0, nblk_link = 0, nblk_site = 0, nblk_lw = 0;
    // Lattice groups of the sweep schedule: group g holds lattices
    // [grp_first[g], grp_first[g + 1]) and its phase blocks are counted by
    // d_bbeg_grp + grp_off[g] (starting at 0).
    std::vector<int> grp_first, grp_off, grp_nblk;
    int* d_bbeg_grp = nullptr;
    double* d_partials = nullptr;
    double* d_out = nullptr;  // reduction results
    // plaquette site values written by the last overrelaxation pass of a
    // sweep (3 Vh doubles per lattice), their block tables and partials
    double* d_psite = nullptr;
    size_t psite_cap = 0;
    int* d_bbeg_psite = nullptr;
    double* d_partials2 = nullptr;
    int nblk_psite = 0;
    int out_cap = 0;
    uint64_t* d_sweep = nullptr;
    unsigned long long* d_exh = nullptr;  // exhausted heat-bath draws, one counter per lattice
    std::vector<LatDesc> host_descs;
    std::vector<int> bbeg_phase_h, bbeg_link_h, bbeg_site_h, bbeg_lw_h;

    void release()
    {
        hipFree(d_descs);
        hipFree(d_bbeg_phase);
        hipFree(d_bbeg_link);
        hipFree(d_bbeg_site);
        hipFree(d_bbeg_lw);
        hipFree(d_bbeg_grp);
        hipFree(d_partials);
        hipFree(d_out);
        hipFree(d_sweep);
        hipFree(d_exh);
        hipFree(d_psite);
        hipFree(d_bbeg_psite);
        hipFree(d_partials2);
        d_psite = d_partials2 = nullptr;
        d_bbeg_psite = nullptr;
        psite_cap = 0;
        nblk_psite = 0;
        d_descs = nullptr;
        d_bbeg_phase = d_bbeg_link = d_bbeg_site = d_bbeg_lw = d_bbeg_grp = nullptr;
        grp_first.clear();
        grp_off.clear();
        grp_nblk.clear();
        d_partials = d_out = nullptr;
        d_sweep = nullptr;
        d_exh = nullptr;
        out_cap = 0;
    }
    Grid grid_phase() const { return Grid{ d_descs, d_bbeg_phase, nlat, nblk_phase, phase_block, remap }; }
    int ngroups() const { return (int)grp_nblk.size(); }
    Grid grid_phase_group(int g) const
    {
        return Grid{ d_descs + grp_first[g], d_bbeg_grp + grp_off[g], grp_first[g + 1] - grp_first[g], grp_nblk[g],
                     phase_block, remap };
    }
    Grid grid_link(const LatDesc* descs = nullptr) const
    {
        return Grid{ descs ? descs : d_descs, d_bbeg_link, nlat, nblk_link, 256, 1 };
    }
    Grid grid_site(const LatDesc* descs = nullptr) const
    {
        return Grid{ descs ? descs : d_descs, d_bbeg_site, nlat, nblk_site, 256, 1 };
    }
    // all 4V links, four directions of 64 sites per block (link_walk)
    Grid grid_lw(const LatDesc* descs = nullptr) const
    {
        return Grid{ descs ? descs : d_descs, d_bbeg_lw, nlat, nblk_lw, 256, 1 };
    }
    // plaquette site values, 1024 per block
    Grid grid_psite() const { return Grid{ d_descs, d_bbeg_psite, nlat, nblk_psite, 256, 0 }; }
};

struct su3_field_s {
    int L[4];
    int V = 0, Vh = 0;
    int prec = 0, NC = 18;
    size_t cs = 0, cs8 = 0, bytes = 0, bytes8 = 0;
    void* data = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    // scratch
    void* alt[3] = { nullptr, nullptr, nullptr };
    void* aux8 = nullptr;
    LatDesc* d_extra = nullptr;  // 8 descriptor variants (HMC / flow ping-pong)
    Plan plan;                    // single-lattice tables
    bool plan_ready = false;
    int64_t last_exhausted = 0;
    Geo geo() const
    {
        Geo g;
        for (int m = 0; m < 4; m++) g.L[m] = L[m];
        g.h0 = L[0] / 2;
        g.Vh = Vh;
        return g;
    }
};

static int32_t check_dims(const int32_t* dims)
{
    if (!dims) return fail(SU3_ERR_ARG, "dims is NULL");
    long long V = 1;
    for (int m = 0; m < 4; m++) {
        if (dims[m] < 2 || (dims[m] & 1))
            return fail(SU3_ERR_SHAPE, "every extent must be even and >= 2 (dims[" + std::to_string(m) +
                                           "] = " + std::to_string(dims[m]) + ")");
        V *= dims[m];
        if (V > (1LL << 28)) return fail(SU3_ERR_SHAPE, "volume exceeds 2^28 sites");
    }
    return SU3_OK;
}

static void layout(const int32_t* dims, int prec, size_t& cs, size_t& cs8, size_t& bytes, size_t& bytes8)
{
    long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    const size_t Vh = (size_t)(V / 2);
    const size_t rb = prec_real_bytes(prec);
    cs = slab_bytes(Vh, prec_ncomp(prec), rb);
    cs8 = slab_bytes(Vh, 8, rb);
    bytes = 8 * cs;
    bytes8 = 8 * cs8;
}

static int32_t check_field(su3_field f)
{
    if (!f) return fail(SU3_ERR_ARG, "field handle is NULL");
    return SU3_OK;
}

static LatDesc base_desc(const su3_field_s* f)
{
    LatDesc d;
    memset(&d, 0, sizeof d);
    d.U = f->data;
    d.aux = f->aux8;
    d.aux2 = f->alt[0];
    d.cs = f->cs;
    d.cs8 = f->cs8;
    d.g = f->geo();
    d.tile[0] = largest_divisor_upto(f->L[1], 16);  // plans replace it with the launch choice
    d.tile[1] = largest_divisor_upto(f->L[2], 8);
    d.tile[2] = largest_divisor_upto(f->L[3], 4);
    d.mtile[0] = largest_divisor_upto(f->L[1], 8);
    d.mtile[1] = largest_divisor_upto(f->L[2], 8);
    d.mtile[2] = largest_divisor_upto(f->L[3], 4);
    return d;
}

static int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Build or rebuild the device tables of a plan for the given fields.
// Batches are swept group by group, each group's links at most this many
// bytes (a lattice larger than that is a group of its own), so that a group
// stays resident in the 256 MB last-level cache across the phases of a sweep.
// 0: the whole batch is one group.
static size_t g_group_bytes = (size_t)224 << 20;

// With psite the plan also holds the buffers that let the sweeps form the
// plaquette in their last overrelaxation pass.
static int32_t plan_build(Plan& p, const std::vector<su3_field_s*>& fs, const LaunchCfg& cfg, int out_cap,
                          hipStream_t st, bool psite = false)
{
    const bool shape_change = p.nlat != (int)fs.size();
    if (shape_change) p.release();
    const int phase_block = cfg.block;
    p.nlat = (int)fs.size();
    p.prec = fs[0]->prec;
    p.cfg = cfg;
    p.phase_block = phase_block;
    p.remap = cfg.remap;
    p.host_descs.clear();
    p.bbeg_phase_h.assign(1, 0);
    p.bbeg_link_h.assign(1, 0);
    p.bbeg_site_h.assign(1, 0);
    p.bbeg_lw_h.assign(1, 0);
    for (auto* f : fs) {
        LatDesc d = base_desc(f);
        d.tile[0] = largest_divisor_upto(f->L[1], cfg.ty);
        d.tile[1] = largest_divisor_upto(f->L[2], cfg.tz);
        d.tile[2] = largest_divisor_upto(f->L[3], cfg.tt);
        p.host_descs.push_back(d);
        p.bbeg_phase_h.push_back(p.bbeg_phase_h.back() + ceil_div(f->Vh, phase_block));
        p.bbeg_link_h.push_back(p.bbeg_link_h.back() + ceil_div(8LL * f->Vh, 256));
        p.bbeg_site_h.push_back(p.bbeg_site_h.back() + ceil_div(2LL * f->Vh, 256));
        p.bbeg_lw_h.push_back(p.bbeg_lw_h.back() + 2 * ceil_div(f->Vh, 64));
    }
    std::vector<int> bbeg_psite_h(1, 0);
    size_t psite_n = 0;
    for (auto* f : fs) {
        bbeg_psite_h.push_back(bbeg_psite_h.back() + ceil_div(3LL * f->Vh, 1024));
        psite_n += 3 * (size_t)f->Vh;
    }
    p.nblk_phase = p.bbeg_phase_h.back();
    p.nblk_link = p.bbeg_link_h.back();
    p.nblk_site = p.bbeg_site_h.back();
    p.nblk_lw = p.bbeg_lw_h.back();
    // lattice groups (consecutive lattices, at most g_group_bytes of links each)
    std::vector<int> gb;
    p.grp_first.assign(1, 0);
    p.grp_off.clear();
    p.grp_nblk.clear();
    {
        size_t acc = 0;
        for (int i = 0; i < p.nlat; i++) {
            if (i > p.grp_first.back() && g_group_bytes > 0 && acc + fs[i]->bytes > g_group_bytes) {
                p.grp_first.push_back(i);
                acc = 0;
            }
            acc += fs[i]->bytes;
        }
        p.grp_first.push_back(p.nlat);
        for (int g = 0; g + 1 < (int)p.grp_first.size(); g++) {
            const int a = p.grp_first[g], e = p.grp_first[g + 1];
            p.grp_off.push_back((int)gb.size());
            for (int i = a; i <= e; i++) gb.push_back(p.bbeg_phase_h[i] - p.bbeg_phase_h[a]);
            p.grp_nblk.push_back(p.bbeg_phase_h[e] - p.bbeg_phase_h[a]);
        }
    }
    if (!p.d_descs) {
        HIPCHK(hipMalloc(&p.d_descs, sizeof(LatDesc) * p.nlat));
        HIPCHK(hipMalloc(&p.d_bbeg_phase, sizeof(int) * (p.nlat + 1)));
        HIPCHK(hipMalloc(&p.d_bbeg_link, sizeof(int) * (p.nlat + 1)));
        HIPCHK(hipMalloc(&p.d_bbeg_site, sizeof(int) * (p.nlat + 1)));
        HIPCHK(hipMalloc(&p.d_bbeg_lw, sizeof(int) * (p.nlat + 1)));
        HIPCHK(hipMalloc(&p.d_bbeg_grp, sizeof(int) * (2 * p.nlat + 1)));
        // up to 5 classes of site partials (Wilson loop classes) or one per link block
        HIPCHK(hipMalloc(&p.d_partials, sizeof(double) * std::max({ 5 * p.nblk_site, p.nblk_link, p.nblk_lw })));
        HIPCHK(hipMalloc(&p.d_sweep, sizeof(uint64_t)));
        HIPCHK(hipMalloc(&p.d_exh, sizeof(unsigned long long) * p.nlat));
    }
    if (out_cap > p.out_cap) {
        hipFree(p.d_out);
        p.d_out = nullptr;
        HIPCHK(hipMalloc(&p.d_out, sizeof(double) * out_cap));
        p.out_cap = out_cap;
    }
    if (psite && p.psite_cap < psite_n) {
        hipFree(p.d_psite);
        hipFree(p.d_bbeg_psite);
        hipFree(p.d_partials2);
        p.d_psite = p.d_partials2 = nullptr;
        p.d_bbeg_psite = nullptr;
        p.psite_cap = 0;
        HIPCHK(hipMalloc(&p.d_psite, sizeof(double) * psite_n));
        HIPCHK(hipMalloc(&p.d_bbeg_psite, sizeof(int) * (p.nlat + 1)));
        HIPCHK(hipMalloc(&p.d_partials2, sizeof(double) * bbeg_psite_h.back()));
        p.psite_cap = psite_n;
    }
    if (p.d_psite) {
        p.nblk_psite = bbeg_psite_h.back();
        size_t off = 0;
        for (int i = 0; i < p.nlat; i++) {
            p.host_descs[i].psite = p.d_psite + off;
            off += 3 * (size_t)fs[i]->Vh;
        }
        HIPCHK(upload_ints(p.d_bbeg_psite, bbeg_psite_h, st));
    }
    HIPCHK(upload_descs(p.d_descs, p.host_descs, st));
    HIPCHK(upload_ints(p.d_bbeg_phase, p.bbeg_phase_h, st));
    HIPCHK(upload_ints(p.d_bbeg_link, p.bbeg_link_h, st));
    HIPCHK(upload_ints(p.d_bbeg_site, p.bbeg_site_h, st));
    HIPCHK(upload_ints(p.d_bbeg_lw, p.bbeg_lw_h, st));
    HIPCHK(upload_ints(p.d_bbeg_grp, gb, st));
    return SU3_OK;
}

// ---------------------------------------------------------------------------
// Launch configuration, autotuning and profiling state.
// ---------------------------------------------------------------------------
static std::mutex g_mu;
static int g_forced_block = 0, g_forced_remap = 1;
static int g_forced_tile[3] = { 0, 0, 0 };
static bool g_tile_forced = false;
static bool g_autotune = false;
static std::map<std::string, LaunchCfg> g_tuned;
static bool g_profile = false;

static double g_prof_ms[3] = { 0, 0, 0 };
static long long g_prof_n[3] = { 0, 0, 0 };
static std::vector<hipEvent_t> g_events;

static std::string shape_key(const std::vector<su3_field_s*>& fs)
{
    std::string k = std::to_string(fs[0]->prec);
    for (auto* f : fs) k += ":" + std::to_string(f->L[0]) + "x" + std::to_string(f->L[1]) + "x" +
                            std::to_string(f->L[2]) + "x" + std::to_string(f->L[3]);
    return k;
}

// Default tile: 8 x 8 x 8 sites in (y, z, t) when the extents allow it (with
// XCD-contiguous block ranges each XCD then sweeps a compact region; at 32^4 a
// 12-real overrelaxation phase fetched 2 % less than with 16 x 8 x 4).
static LaunchCfg default_cfg()
{
    LaunchCfg c;
    c.block = 256;
    c.remap = 1;
    c.ty = 8;
    c.tz = 8;
    c.tt = 8;
    return c;
}

static LaunchCfg launch_choice(const std::vector<su3_field_s*>& fs)
{
    std::lock_guard<std::mutex> lk(g_mu);
    LaunchCfg c = default_cfg();
    auto it = g_tuned.find(shape_key(fs));
    if (it != g_tuned.end()) c = it->second;
    if (g_forced_block > 0) {
        c.block = g_forced_block;
        c.remap = g_forced_remap;
    }
    if (g_tile_forced) {
        c.ty = g_forced_tile[0];
        c.tz = g_forced_tile[1];
        c.tt = g_forced_tile[2];
    }
    return c;
}

static int32_t ensure_events(size_t n)
{
    while (g_events.size() < n) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        g_events.push_back(e);
    }
    return SU3_OK;
}

// ---------------------------------------------------------------------------
// The sweep schedule, shared by the eager single-lattice path, the graph
// capture of batches and the autotuner.  Enqueues n_sweeps sweeps on st.
// ---------------------------------------------------------------------------
struct SweepOpts {
    int n_or, n_hits, max_tries, reunit_every, sampler;
    bool record;
};

// Profiling: HIP events around a run of consecutive launches of one kind
// (the heat-bath pass, the overrelaxation passes of a lattice group, the
// plaquette), so that the average per launch carries no per-launch event
// overhead.
struct ProfRun {
    int ev, kind, count;
};

struct ProfMark {
    std::vector<ProfRun>* marks;
    hipStream_t st;
    int ev = -1;
    int32_t begin()
    {
        if (!marks) return SU3_OK;
        ev = (int)marks->size() * 2;
        int32_t rc = ensure_events((size_t)ev + 2);
        if (rc) return rc;
        HIPCHK(hipEventRecord(g_events[ev], st));
        return SU3_OK;
    }
    int32_t end(int kind, int count)
    {
        if (!marks) return SU3_OK;
        HIPCHK(hipEventRecord(g_events[ev + 1], st));
        marks->push_back({ ev, kind, count });
        return SU3_OK;
    }
};

static int32_t read_marks(const std::vector<ProfRun>& marks)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& m : marks) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, g_events[m.ev], g_events[m.ev + 1]));
        g_prof_ms[m.kind] += ms;
        g_prof_n[m.kind] += m.count;
    }
    return SU3_OK;
}

static int32_t enqueue_sweeps(const Plan& p, int n_sweeps, const SweepOpts& o, hipStream_t st,
                              std::vector<ProfRun>* prof_marks)
{
    const HbArgs hb{ o.n_hits, o.max_tries, o.sampler };
    // a plan without group tables sweeps all its lattices as one group
    const int ng = std::max(1, p.ngroups());
    // the plaquette is formed in the last overrelaxation pass when the plan
    // has the buffers for it
    const bool fused = o.record && p.d_psite && o.n_or >= 1;
    // fp32 and 12-real links leave every sweep re-orthonormalized in fp64 by
    // the stores of its last pass, which leaves nothing for the
    // reunitarization every reunit_every sweeps to do: it runs on fp64
    // fields only (and with it the fresh plaquette of such a sweep)
    const int every = p.prec == PREC_F64 ? o.reunit_every : 0;
    int32_t rc;
    for (int k = 0; k < n_sweeps; k++) {
        // Lattices are independent: each group runs its whole sweep before the
        // next group starts, so its links stay cached between phases.
        for (int grp = 0; grp < ng; grp++) {
            const Grid gph = ng > 1 ? p.grid_phase_group(grp) : p.grid_phase();
            unsigned long long* exh = p.d_exh + (ng > 1 ? p.grp_first[grp] : 0);
            ProfMark pm{ prof_marks, st };
            for (int pass = 0; pass <= o.n_or; pass++) {
                // bits of the phase kernels: 1 overrelaxation, 2 plaquette site
                // values, 4 fp64 re-orthonormalization of fp32 stores (last pass)
                const int kind = (pass == 0 ? 0 : 1) | (pass == o.n_or ? 4 : 0);
                if (pass <= 1 && (rc = pm.begin())) return rc;
                for (int mu = 0; mu < 4; mu++)
                    for (int par = 0; par < 2; par++) {
                        const int kk = kind | ((fused && pass == o.n_or && par == 1 && mu >= 1) ? 2 : 0);
                        HIPCHK(launch_phase(p.prec, kk, gph, mu, par, p.d_sweep, k, hb, pass == 0 ? exh : nullptr,
                                            st));
                    }
                if (pass == 0 && (rc = pm.end(0, 8))) return rc;
                if (pass == o.n_or && pass > 0 && (rc = pm.end(1, 8 * o.n_or))) return rc;
            }
        }
        if (every > 0) HIPCHK(launch_reunit(p.prec, p.grid_link(), p.d_sweep, k, every, st));
        if (o.record) {
            ProfMark pm{ prof_marks, st };
            if ((rc = pm.begin())) return rc;
            if (fused) {
                // site values of the last pass; in a sweep that reunitarizes
                // the plaquette is taken afresh from the reunitarized links
                HIPCHK(launch_psite_partial(p.grid_psite(), p.d_partials2, st));
                if (every > 0)
                    HIPCHK(launch_plaq_partial_gated(p.prec, p.grid_site(), p.d_partials, p.d_sweep, k, every,
                                                     st));
                if ((rc = pm.end(2, 1))) return rc;
                HIPCHK(launch_reduce_pick(p.nlat, p.d_bbeg_site, p.d_partials, p.d_bbeg_psite, p.d_partials2,
                                          p.d_sweep, k, every, p.d_out, 1, k * p.nlat, st));
            } else {
                HIPCHK(launch_plaq_partial(p.prec, p.grid_site(), p.d_partials, st));
                if ((rc = pm.end(2, 1))) return rc;
                HIPCHK(launch_reduce_final(p.grid_site(), p.d_partials, p.d_out, 1, k * p.nlat, st));
            }
        }
    }
    return SU3_OK;
}

static int32_t validate_hb(const su3_hb_params* pp, SweepOpts& o)
{
    su3_hb_params d{ 4, 1, 64, 10, SU3_SAMPLER_KP };
    const su3_hb_params& p = pp ? *pp : d;
    if (p.n_or < 0 || p.n_or > 1000) return fail(SU3_ERR_ARG, "n_or must be in [0, 1000]");
    if (p.n_hb_hits < 1 || p.n_hb_hits > 255) return fail(SU3_ERR_ARG, "n_hb_hits must be in [1, 255]");
    if (p.hb_max_tries < 1 || p.hb_max_tries > 4096) return fail(SU3_ERR_ARG, "hb_max_tries must be in [1, 4096]");
    if (p.reunit_every < 0) return fail(SU3_ERR_ARG, "reunit_every must be >= 0");
    if (p.sampler != SU3_SAMPLER_KP && p.sampler != SU3_SAMPLER_CREUTZ) return fail(SU3_ERR_ARG, "unknown sampler");
    o.n_or = p.n_or;
    o.n_hits = p.n_hb_hits;
    o.max_tries = p.hb_max_tries;
    o.reunit_every = p.reunit_every;
    o.sampler = p.sampler;
    return SU3_OK;
}

// Time each launch shape on scratch fields (cold starts) of the given shapes
// with sweeps of the calling sweep's own couplings and options, and remember
// the fastest for this shape set; the default shape is kept unless another is
// faster by more than 1.5 % (differences below that are run-to-run noise).
// The couplings matter: at beta = 0 every heat-bath trial is rejected, so a
// pass costs several times what it does at the couplings of interest.
static int32_t autotune(const std::vector<su3_field_s*>& fs, const double* betas, const SweepOpts& call,
                        hipStream_t st)
{
    std::vector<su3_field_s> scratch(fs.size());
    std::vector<su3_field_s*> sp;
    int32_t rc = SU3_OK;
    for (size_t i = 0; i < fs.size(); i++) {
        scratch[i] = *fs[i];
        scratch[i].data = nullptr;
        scratch[i].owned = true;
        scratch[i].plan_ready = false;
        scratch[i].plan = Plan();
        if (hipMalloc(&scratch[i].data, fs[i]->bytes) != hipSuccess) {
            rc = fail(SU3_ERR_NOMEM, "autotune scratch allocation failed");
            break;
        }
        sp.push_back(&scratch[i]);
    }
    Plan p;
    std::vector<LaunchCfg> cand{ default_cfg() };
    const int blocks[] = { 128, 256, 512 };
    const int tiles[][3] = { { 0, 0, 1 }, { 16, 8, 4 }, { 16, 16, 4 }, { 8, 8, 8 }, { 16, 8, 8 }, { 32, 8, 4 }, { 8, 8, 16 } };
    for (int remap = 0; remap < 2; remap++)
        for (int b : blocks)
            for (auto& t : tiles) {
                LaunchCfg c;
                c.block = b;
                c.remap = remap;
                c.ty = t[0];
                c.tz = t[1];
                c.tt = t[2];
                const LaunchCfg d = default_cfg();
                if (c.block == d.block && c.remap == d.remap && c.ty == d.ty && c.tz == d.tz && c.tt == d.tt) continue;
                cand.push_back(c);
            }
    float best = 1e30f, t_default = 1e30f;
    LaunchCfg bestc = default_cfg();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(SU3_ERR_HIP, "event creation failed");
    for (size_t ci = 0; ci < cand.size() && !rc; ci++) {
        {
            rc = plan_build(p, sp, cand[ci], 1, st);
            if (rc) break;
            for (size_t i = 0; i < sp.size(); i++) {
                p.host_descs[i].seed = 12345u + (uint32_t)i;
                p.host_descs[i].beta = betas[i];
            }
            // every candidate starts from the same cold fields: the cost of a
            // heat-bath pass depends on the field
            if (upload_descs(p.d_descs, p.host_descs, st) != hipSuccess ||
                launch_init(p.prec, 0, p.grid_link(), st) != hipSuccess) {
                rc = fail(SU3_ERR_HIP, "autotune init failed");
                break;
            }
            k_set_u64<<<1, 1, 0, st>>>(p.d_sweep, 0);
            SweepOpts o = call;
            o.record = false;
            rc = enqueue_sweeps(p, 1, o, st, nullptr);  // warm-up
            if (rc) break;
            hipEventRecord(e0, st);
            rc = enqueue_sweeps(p, 2, o, st, nullptr);
            if (rc) break;
            hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) {
                rc = fail(SU3_ERR_HIP, "autotune timing failed");
                break;
            }
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            if (ci == 0) t_default = ms;
            if (ms < best) {
                best = ms;
                bestc = cand[ci];
            }
        }
    }
    hipStreamSynchronize(st);
    p.release();
    for (auto& s : scratch) hipFree(s.data);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (rc) return rc;
    if (best > 0.985f * t_default) bestc = default_cfg();
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned[shape_key(fs)] = bestc;
    return SU3_OK;
}

// ---------------------------------------------------------------------------
// Graph cache for batched sweeps.
// ---------------------------------------------------------------------------
struct GraphEntry {
    std::string key;
    std::vector<su3_field_s*> fields;
    Plan plan;
    bool descs_current = false;  // plan.d_descs hold plan.host_descs (only this call writes them)
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t capture = nullptr;
};
static std::vector<GraphEntry*> g_graphs;

static void drop_graph(GraphEntry* g)
{
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    if (g->capture) hipStreamDestroy(g->capture);
    g->plan.release();
    delete g;
}

static void forget_field_graphs(su3_field_s* f)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t i = 0; i < g_graphs.size();) {
        GraphEntry* g = g_graphs[i];
        if (std::find(g->fields.begin(), g->fields.end(), f) != g->fields.end()) {
            hipStreamSynchronize(f->stream);
            drop_graph(g);
            g_graphs.erase(g_graphs.begin() + i);
        } else {
            i++;
        }
    }
}

// ---------------------------------------------------------------------------
// Host Philox (for the Metropolis test) -- the same generator as on device.
// ---------------------------------------------------------------------------
static void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, y1 = (uint32_t)p1;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1, y3 = (uint32_t)p0;
        c[0] = y0;
        c[1] = y1;
        c[2] = y2;
        c[3] = y3;
    }
}

// ---------------------------------------------------------------------------
// Single-field helpers
// ---------------------------------------------------------------------------
static int32_t single_plan(su3_field_s* f, int out_cap, bool psite = false)
{
    std::vector<su3_field_s*> fs{ f };
    const LaunchCfg cfg = launch_choice(fs);
    if (!f->plan_ready || !(f->plan.cfg == cfg) || f->plan.out_cap < out_cap || f->plan.host_descs.empty() ||
        f->plan.host_descs[0].aux != f->aux8 || f->plan.host_descs[0].aux2 != f->alt[0] ||
        (psite && !f->plan.d_psite)) {
        int32_t rc = plan_build(f->plan, fs, cfg, std::max(out_cap, 8), f->stream, psite || f->plan.d_psite);
        if (rc) return rc;
        f->plan_ready = true;
    }
    return SU3_OK;
}

// Descriptor of f carrying its plan's launch tile (single_plan must have run):
// the link walks of the HMC and flow kernels then follow the tuned or forced
// tile, like the phase kernels.
static LatDesc plan_desc(const su3_field_s* f)
{
    LatDesc d = base_desc(f);
    if (!f->plan.host_descs.empty())
        for (int k = 0; k < 3; k++) d.tile[k] = f->plan.host_descs[0].tile[k];
    return d;
}

static int32_t ensure_scratch(su3_field_s* f, bool alts, bool aux, int n_alts = 2)
{
    if (alts) {
        for (int k = 0; k < n_alts; k++)
            if (!f->alt[k] && hipMalloc(&f->alt[k], f->bytes) != hipSuccess)
                return fail(SU3_ERR_NOMEM, "scratch field allocation failed");
    }
    if (aux && !f->aux8 && hipMalloc(&f->aux8, f->bytes8) != hipSuccess)
        return fail(SU3_ERR_NOMEM, "momentum buffer allocation failed");
    if (!f->d_extra && hipMalloc(&f->d_extra, sizeof(LatDesc) * 8) != hipSuccess)
        return fail(SU3_ERR_NOMEM, "descriptor allocation failed");
    f->plan_ready = false;  // descriptors carry the scratch pointers
    return SU3_OK;
}

// result = sum over sites of [1 - (1/3) Re Tr U_p] using descriptor d (on device)
static int32_t action_density_sum(su3_field_s* f, const LatDesc* d, double* out)
{
    Plan& p = f->plan;
    HIPCHK(launch_plaq_partial(f->prec, p.grid_site(d), p.d_partials, f->stream));
    HIPCHK(launch_reduce_final(p.grid_site(d), p.d_partials, p.d_out, 1, 0, f->stream));
    HIPCHK(hipMemcpyAsync(out, p.d_out, sizeof(double), hipMemcpyDeviceToHost, f->stream));
    HIPCHK(hipStreamSynchronize(f->stream));
    return SU3_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free sweeps: the tables, counters, plaquette partials and
// history of one lattice live in a fixed device array instead of per-field
// allocations.  Layout (bytes): descriptor [0, 256), block tables
// [256, 512), sweep index and exhausted-draw counter [512, 768), plaquette
// block partials (one double per 256 sites) [768, 768 + 8 * kNaPartials),
// then the per-sweep sums (kNaMaxRecord doubles).
// ---------------------------------------------------------------------------
constexpr long long kNaMaxSites = 1LL << 24;  // e.g. 64^4
constexpr int kNaMaxRecord = 4096;            // sweeps with a plaquette history per call
constexpr size_t kNaPartials = (size_t)(kNaMaxSites / 256);
constexpr size_t kNaOffDesc = 0, kNaOffInts = 256, kNaOffCounters = 512, kNaOffPartials = 768;
constexpr size_t kNaOffOut = kNaOffPartials + sizeof(double) * kNaPartials;
constexpr size_t kNaBytes = kNaOffOut + sizeof(double) * kNaMaxRecord;
static_assert(sizeof(LatDesc) <= kNaOffInts - kNaOffDesc, "descriptor slot too small");

// Each GPU the library runs on holds one copy until the process ends.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

static std::mutex g_na_mu;
constexpr int kNaMaxDevices = 64;
static void* g_na_ptr[kNaMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device (the array's name is not a device address in host code).
static int32_t na_scratch(unsigned char** out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(SU3_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SU3_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_na_ptr[dev] = ptr;
    }
    *out = (unsigned char*)g_na_ptr[dev];
    return SU3_OK;
}

// Launch shape of the allocation-free sweeps: the default, or the shape
// forced by su3_set_launch / su3_set_tile (autotuned shapes are not used).
static LaunchCfg na_launch_cfg()
{
    std::lock_guard<std::mutex> lk(g_mu);
    LaunchCfg c = default_cfg();
    if (g_forced_block > 0) {
        c.block = g_forced_block;
        c.remap = g_forced_remap;
    }
    if (g_tile_forced) {
        c.ty = g_forced_tile[0];
        c.tz = g_forced_tile[1];
        c.tt = g_forced_tile[2];
    }
    return c;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* su3_last_error(void) { return g_err.c_str(); }

int32_t su3_field_bytes(const int32_t dims[4], int32_t prec, size_t* out)
{
    int32_t rc = check_dims(dims);
    if (rc) return rc;
    if (prec < 0 || prec > 2) return fail(SU3_ERR_ARG, "unknown precision");
    if (!out) return fail(SU3_ERR_ARG, "out is NULL");
    size_t cs, cs8, b, b8;
    layout(dims, prec, cs, cs8, b, b8);
    *out = b;
    return SU3_OK;
}

static int32_t make_field(const int32_t dims[4], int32_t prec, void* ptr, size_t nbytes, bool own, void* stream,
                          su3_field* out)
{
    int32_t rc = check_dims(dims);
    if (rc) return rc;
    if (prec < 0 || prec > 2) return fail(SU3_ERR_ARG, "unknown precision");
    if (!out) return fail(SU3_ERR_ARG, "out is NULL");
    su3_field_s* f = new su3_field_s();
    for (int m = 0; m < 4; m++) f->L[m] = dims[m];
    f->V = dims[0] * dims[1] * dims[2] * dims[3];
    f->Vh = f->V / 2;
    f->prec = prec;
    f->NC = prec_ncomp(prec);
    layout(dims, prec, f->cs, f->cs8, f->bytes, f->bytes8);
    f->stream = (hipStream_t)stream;
    if (own) {
        if (hipMalloc(&f->data, f->bytes) != hipSuccess) {
            delete f;
            return fail(SU3_ERR_NOMEM, "field allocation of " + std::to_string(f->bytes) + " bytes failed");
        }
        f->owned = true;
    } else {
        if (!ptr) {
            delete f;
            return fail(SU3_ERR_ARG, "dev_ptr is NULL");
        }
        if (nbytes < f->bytes) {
            size_t need = f->bytes;
            delete f;
            return fail(SU3_ERR_ARG, "wrapped buffer too small: need " + std::to_string(need) + " bytes");
        }
        if (((uintptr_t)ptr) & 255) {
            delete f;
            return fail(SU3_ERR_ARG, "wrapped buffer must be 256-byte aligned");
        }
        f->data = ptr;
        f->owned = false;
    }
    *out = f;
    return SU3_OK;
}

int32_t su3_field_create(const int32_t dims[4], int32_t prec, void* hip_stream, su3_field* out)
{
    return make_field(dims, prec, nullptr, 0, true, hip_stream, out);
}

int32_t su3_field_wrap(const int32_t dims[4], int32_t prec, void* dev_ptr, size_t bytes, void* hip_stream,
                       su3_field* out)
{
    return make_field(dims, prec, dev_ptr, bytes, false, hip_stream, out);
}

int32_t su3_field_destroy(su3_field f)
{
    if (!f) return SU3_OK;
    forget_field_graphs(f);
    hipStreamSynchronize(f->stream);
    f->plan.release();
    if (f->owned) hipFree(f->data);
    hipFree(f->alt[0]);
    hipFree(f->alt[1]);
    hipFree(f->alt[2]);
    hipFree(f->aux8);
    hipFree(f->d_extra);
    delete f;
    return SU3_OK;
}

int32_t su3_field_set_stream(su3_field f, void* hip_stream)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    f->stream = (hipStream_t)hip_stream;
    return SU3_OK;
}

int32_t su3_field_info(su3_field f, int32_t dims[4], int32_t* prec, size_t* bytes)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (dims)
        for (int m = 0; m < 4; m++) dims[m] = f->L[m];
    if (prec) *prec = f->prec;
    if (bytes) *bytes = f->bytes;
    return SU3_OK;
}

int32_t su3_init_cold(su3_field f)
{
    int32_t rc = check_field(f);
    if (!rc) rc = single_plan(f, 1);
    if (rc) return rc;
    HIPCHK(launch_init(f->prec, 0, f->plan.grid_link(), f->stream));
    return SU3_OK;
}

int32_t su3_init_hot(su3_field f, uint32_t seed, uint32_t lattice_id)
{
    int32_t rc = check_field(f);
    if (!rc) rc = single_plan(f, 1);
    if (rc) return rc;
    std::vector<LatDesc> d{ f->plan.host_descs[0] };
    d[0].seed = seed;
    d[0].lid = lattice_id;
    HIPCHK(upload_descs(f->plan.d_descs, d, f->stream));
    HIPCHK(launch_init(f->prec, 1, f->plan.grid_link(), f->stream));
    return SU3_OK;
}

int32_t su3_field_to_host(su3_field f, double* out)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!out) return fail(SU3_ERR_ARG, "out is NULL");
    const size_t n = (size_t)f->V * 72 * sizeof(double);
    double* stage = nullptr;
    HIPCHK(hipMalloc(&stage, n));
    hipError_t e = launch_to_aos(f->prec, nullptr, f->geo(), f->data, f->cs, stage, f->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, stage, n, hipMemcpyDeviceToHost, f->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    hipFree(stage);
    if (e != hipSuccess) return fail(SU3_ERR_HIP, std::string("to_host: ") + hipGetErrorString(e));
    return SU3_OK;
}

int32_t su3_field_from_host(su3_field f, const double* in)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!in) return fail(SU3_ERR_ARG, "in is NULL");
    const size_t n = (size_t)f->V * 72 * sizeof(double);
    double* stage = nullptr;
    HIPCHK(hipMalloc(&stage, n));
    hipError_t e = hipMemcpyAsync(stage, in, n, hipMemcpyHostToDevice, f->stream);
    if (e == hipSuccess) e = launch_from_aos(f->prec, f->geo(), f->data, f->cs, stage, f->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    hipFree(stage);
    if (e != hipSuccess) return fail(SU3_ERR_HIP, std::string("from_host: ") + hipGetErrorString(e));
    return SU3_OK;
}

int32_t su3_field_copy(su3_field dst, su3_field src)
{
    int32_t rc = check_field(dst);
    if (!rc) rc = check_field(src);
    if (rc) return rc;
    for (int m = 0; m < 4; m++)
        if (dst->L[m] != src->L[m]) return fail(SU3_ERR_SHAPE, "copy between fields of different shapes");
    if (dst->stream != src->stream) HIPCHK(hipStreamSynchronize(src->stream));
    HIPCHK(launch_convert(dst->prec, dst->data, dst->cs, src->prec, src->data, src->cs, src->Vh, dst->stream));
    return SU3_OK;
}

int32_t su3_sweep_hb_or(su3_field f, double beta, uint32_t seed, uint32_t lattice_id, uint64_t first_sweep,
                        int32_t n_sweeps, const su3_hb_params* pp, double* plaq_hist)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    SweepOpts o;
    if ((rc = validate_hb(pp, o))) return rc;
    if (n_sweeps < 0) return fail(SU3_ERR_ARG, "n_sweeps must be >= 0");
    if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(SU3_ERR_ARG, "beta must be finite and >= 0");
    o.record = plaq_hist != nullptr;
    if (g_autotune) {
        std::vector<su3_field_s*> fs{ f };
        bool have;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            have = g_tuned.count(shape_key(fs)) > 0;
        }
        if (!have && (rc = autotune(fs, &beta, o, f->stream))) return rc;
    }
    if ((rc = single_plan(f, std::max(1, n_sweeps), o.record))) return rc;
    Plan& p = f->plan;
    std::vector<LatDesc> d{ p.host_descs[0] };
    d[0].beta = beta;
    d[0].seed = seed;
    d[0].lid = lattice_id;
    HIPCHK(upload_descs(p.d_descs, d, f->stream));
    k_set_u64<<<1, 1, 0, f->stream>>>(p.d_sweep, first_sweep);
    k_zero_u64<<<1, 64, 0, f->stream>>>(p.d_exh, 1);
    HIPCHK(hipGetLastError());
    std::vector<ProfRun> marks;
    const bool prof = g_profile;
    if ((rc = enqueue_sweeps(p, n_sweeps, o, f->stream, prof ? &marks : nullptr))) return rc;
    unsigned long long ex = 0;
    HIPCHK(hipMemcpyAsync(&ex, p.d_exh, sizeof ex, hipMemcpyDeviceToHost, f->stream));
    std::vector<double> h;
    if (o.record && n_sweeps > 0) {
        h.resize(n_sweeps);
        HIPCHK(hipMemcpyAsync(h.data(), p.d_out, sizeof(double) * n_sweeps, hipMemcpyDeviceToHost, f->stream));
    }
    HIPCHK(hipStreamSynchronize(f->stream));
    f->last_exhausted = (int64_t)ex;
    for (int k = 0; k < (int)h.size(); k++) plaq_hist[k] = 1.0 - h[k] / (6.0 * f->V);
    if (prof && (rc = read_marks(marks))) return rc;
    return SU3_OK;
}

int32_t su3_sweep_hb_or_noalloc(su3_field f, double beta, uint32_t seed, uint32_t lattice_id, uint64_t first_sweep,
                                int32_t n_sweeps, const su3_hb_params* pp, double* plaq_hist)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    SweepOpts o;
    if ((rc = validate_hb(pp, o))) return rc;
    if (n_sweeps < 0) return fail(SU3_ERR_ARG, "n_sweeps must be >= 0");
    if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(SU3_ERR_ARG, "beta must be finite and >= 0");
    if ((long long)f->V > kNaMaxSites)
        return fail(SU3_ERR_UNSUPPORTED, "su3_sweep_hb_or_noalloc takes at most 2^24 sites (this field has " +
                                             std::to_string(f->V) + ")");
    o.record = plaq_hist != nullptr;
    if (o.record && n_sweeps > kNaMaxRecord)
        return fail(SU3_ERR_ARG, "su3_sweep_hb_or_noalloc records at most 4096 sweeps per call");
    unsigned char* base = nullptr;
    if ((rc = na_scratch(&base))) return rc;
    hipStream_t st = f->stream;

    // tables of one lattice, written by kernels into the scratch array
    const LaunchCfg cfg = na_launch_cfg();
    LatDesc d = base_desc(f);
    d.tile[0] = largest_divisor_upto(f->L[1], cfg.ty);
    d.tile[1] = largest_divisor_upto(f->L[2], cfg.tz);
    d.tile[2] = largest_divisor_upto(f->L[3], cfg.tt);
    d.beta = beta;
    d.seed = seed;
    d.lid = lattice_id;
    Plan p;  // views into the scratch array; it owns nothing and is never released
    p.nlat = 1;
    p.prec = f->prec;
    p.cfg = cfg;
    p.phase_block = cfg.block;
    p.remap = cfg.remap;
    p.nblk_phase = ceil_div(f->Vh, cfg.block);
    p.nblk_link = ceil_div(8LL * f->Vh, 256);
    p.nblk_site = ceil_div(2LL * f->Vh, 256);
    p.nblk_lw = 2 * ceil_div(f->Vh, 64);
    p.d_descs = (LatDesc*)(base + kNaOffDesc);
    int* ints = (int*)(base + kNaOffInts);
    p.d_bbeg_phase = ints;
    p.d_bbeg_link = ints + 2;
    p.d_bbeg_site = ints + 4;
    p.d_bbeg_lw = ints + 6;
    p.d_sweep = (uint64_t*)(base + kNaOffCounters);
    p.d_exh = (unsigned long long*)(base + kNaOffCounters + 8);
    p.d_partials = (double*)(base + kNaOffPartials);
    p.d_out = (double*)(base + kNaOffOut);
    p.out_cap = kNaMaxRecord;
    {
        DescPack dp;
        memset(&dp, 0, sizeof dp);
        dp.n = 1;
        dp.d[0] = d;
        k_fill_descs<<<1, 64, 0, st>>>(dp, p.d_descs);
        IntPack ip;
        memset(&ip, 0, sizeof ip);
        ip.n = 8;
        const int v[8] = { 0, p.nblk_phase, 0, p.nblk_link, 0, p.nblk_site, 0, p.nblk_lw };
        for (int k = 0; k < 8; k++) ip.v[k] = v[k];
        k_fill_ints<<<1, 64, 0, st>>>(ip, ints);
    }
    // the array keeps the previous call's contents: reset what starts at zero
    k_set_u64<<<1, 1, 0, st>>>(p.d_sweep, first_sweep);
    k_zero_u64<<<1, 64, 0, st>>>(p.d_exh, 1);
    HIPCHK(hipGetLastError());
    if ((rc = enqueue_sweeps(p, n_sweeps, o, st, nullptr))) return rc;
    unsigned long long ex = 0;
    HIPCHK(hipMemcpyAsync(&ex, p.d_exh, sizeof ex, hipMemcpyDeviceToHost, st));
    if (o.record && n_sweeps > 0)
        HIPCHK(hipMemcpyAsync(plaq_hist, p.d_out, sizeof(double) * n_sweeps, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    f->last_exhausted = (int64_t)ex;
    if (o.record)
        for (int k = 0; k < n_sweeps; k++) plaq_hist[k] = 1.0 - plaq_hist[k] / (6.0 * f->V);
    return SU3_OK;
}

int32_t su3_batch_sweep_hb_or(const su3_field* fs, int32_t n, const double* betas, const uint32_t* seeds,
                              const uint32_t* lattice_ids, uint64_t first_sweep, int32_t n_sweeps,
                              const su3_hb_params* pp, double* plaq_out)
{
    if (!fs || n <= 0) return fail(SU3_ERR_ARG, "need at least one field");
    if (!betas || !seeds || !lattice_ids) return fail(SU3_ERR_ARG, "betas, seeds and lattice_ids are required");
    if (n_sweeps < 0) return fail(SU3_ERR_ARG, "n_sweeps must be >= 0");
    SweepOpts o;
    int32_t rc = validate_hb(pp, o);
    if (rc) return rc;
    o.record = plaq_out != nullptr;
    std::vector<su3_field_s*> v;
    for (int i = 0; i < n; i++) {
        if (!fs[i]) return fail(SU3_ERR_ARG, "NULL field in batch");
        if (fs[i]->prec != fs[0]->prec) return fail(SU3_ERR_UNSUPPORTED, "a batch must share one precision");
        if (fs[i]->stream != fs[0]->stream) return fail(SU3_ERR_ARG, "a batch must share one stream");
        if (!(betas[i] >= 0.0) || !std::isfinite(betas[i])) return fail(SU3_ERR_ARG, "beta must be finite and >= 0");
        for (int j = 0; j < i; j++)
            if (fs[j] == fs[i]) return fail(SU3_ERR_ARG, "a field appears twice in the batch");
        v.push_back(fs[i]);
    }
    hipStream_t st = fs[0]->stream;
    if (n_sweeps == 0) {
        for (auto* f : v) f->last_exhausted = 0;  // as a single-field call of no sweeps
        return SU3_OK;
    }
    if (g_autotune) {
        bool have;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            have = g_tuned.count(shape_key(v)) > 0;
        }
        if (!have && (rc = autotune(v, betas, o, st))) return rc;
    }
    const LaunchCfg cfg = launch_choice(v);
    std::string key = std::to_string(n_sweeps) + "|" + std::to_string(o.n_or) + "," + std::to_string(o.n_hits) +
                      "," + std::to_string(o.max_tries) + "," + std::to_string(o.reunit_every) + "," +
                      std::to_string(o.sampler) + "," + std::to_string(o.record) + "|" + cfg.str() + "|" +
                      std::to_string(g_group_bytes) + "|";
    for (auto* f : v) {
        char buf[64];
        snprintf(buf, sizeof buf, "%p,", (void*)f);
        key += buf;
    }
    const bool prof = g_profile;
    if (prof) key += "eager";
    GraphEntry* ge = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto* g : g_graphs)
            if (g->key == key) ge = g;
    }
    if (!ge && prof) {
        ge = new GraphEntry();
        ge->key = key;
        ge->fields = v;
        rc = plan_build(ge->plan, v, cfg, n_sweeps * n, st, o.record);
        if (rc) {
            drop_graph(ge);
            return rc;
        }
        std::lock_guard<std::mutex> lk(g_mu);
        g_graphs.push_back(ge);
    }
    if (!ge) {
        ge = new GraphEntry();
        ge->key = key;
        ge->fields = v;
        rc = plan_build(ge->plan, v, cfg, n_sweeps * n, st, o.record);
        if (!rc && hipStreamCreateWithFlags(&ge->capture, hipStreamNonBlocking) != hipSuccess)
            rc = fail(SU3_ERR_HIP, "capture stream creation failed");
        if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = fail(SU3_ERR_HIP, "stream sync failed");
        if (!rc) {
            if (hipStreamBeginCapture(ge->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                rc = fail(SU3_ERR_HIP, "graph capture could not start");
            } else {
                int32_t erc = enqueue_sweeps(ge->plan, n_sweeps, o, ge->capture, nullptr);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(ge->capture, &g);
                ge->graph = g;
                if (erc)
                    rc = erc;
                else if (e != hipSuccess || !g)
                    rc = fail(SU3_ERR_HIP, std::string("graph capture failed: ") + hipGetErrorString(e));
                else if (hipGraphInstantiate(&ge->exec, g, nullptr, nullptr, 0) != hipSuccess)
                    rc = fail(SU3_ERR_HIP, "graph instantiation failed");
            }
        }
        if (rc) {
            drop_graph(ge);
            return rc;
        }
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_graphs.size() >= 16) {
            drop_graph(g_graphs.front());
            g_graphs.erase(g_graphs.begin());
        }
        g_graphs.push_back(ge);
    }
    Plan& p = ge->plan;
    bool same = ge->descs_current;
    for (int i = 0; i < n; i++) {
        same = same && p.host_descs[i].beta == betas[i] && p.host_descs[i].seed == seeds[i] &&
               p.host_descs[i].lid == lattice_ids[i];
        p.host_descs[i].beta = betas[i];
        p.host_descs[i].seed = seeds[i];
        p.host_descs[i].lid = lattice_ids[i];
    }
    if (!same) {
        ge->descs_current = false;
        HIPCHK(upload_descs(p.d_descs, p.host_descs, st));
        ge->descs_current = true;
    }
    k_set_u64<<<1, 1, 0, st>>>(p.d_sweep, first_sweep);
    k_zero_u64<<<1, 256, 0, st>>>(p.d_exh, n);
    HIPCHK(hipGetLastError());
    std::vector<ProfRun> marks;
    if (prof) {
        if ((rc = enqueue_sweeps(p, n_sweeps, o, st, &marks))) return rc;
    } else {
        HIPCHK(hipGraphLaunch(ge->exec, st));
    }
    std::vector<unsigned long long> ex(n, 0ull);
    HIPCHK(hipMemcpyAsync(ex.data(), p.d_exh, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, st));
    std::vector<double> h;
    if (o.record) {
        h.resize((size_t)n_sweeps * n);
        HIPCHK(hipMemcpyAsync(h.data(), p.d_out, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < n; i++) v[i]->last_exhausted = (int64_t)ex[i];
    if (o.record)
        for (int k = 0; k < n_sweeps; k++)
            for (int i = 0; i < n; i++) plaq_out[(size_t)k * n + i] = 1.0 - h[(size_t)k * n + i] / (6.0 * v[i]->V);
    if (prof && (rc = read_marks(marks))) return rc;
    return SU3_OK;
}

int32_t su3_last_exhausted(su3_field f, int64_t* count)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!count) return fail(SU3_ERR_ARG, "count is NULL");
    *count = f->last_exhausted;
    return SU3_OK;
}

int32_t su3_plaquette(su3_field f, double* out)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!out) return fail(SU3_ERR_ARG, "out is NULL");
    if ((rc = single_plan(f, 1))) return rc;
    double s = 0;
    if ((rc = action_density_sum(f, f->plan.d_descs, &s))) return rc;
    *out = 1.0 - s / (6.0 * f->V);
    return SU3_OK;
}

int32_t su3_action(su3_field f, double beta, double* out)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!out) return fail(SU3_ERR_ARG, "out is NULL");
    if ((rc = single_plan(f, 1))) return rc;
    double s = 0;
    if ((rc = action_density_sum(f, f->plan.d_descs, &s))) return rc;
    *out = beta * s;
    return SU3_OK;
}

static int32_t scalar_reduction(su3_field f, int which, double* out)
{
    int32_t rc = single_plan(f, 1);
    if (rc) return rc;
    Plan& p = f->plan;
    if (which == 0)
        HIPCHK(launch_qtop_partial(f->prec, p.grid_site(), p.d_partials, f->stream));
    else
        HIPCHK(launch_energy_partial(f->prec, p.grid_site(), p.d_partials, f->stream));
    HIPCHK(launch_reduce_final(p.grid_site(), p.d_partials, p.d_out, 1, 0, f->stream));
    HIPCHK(hipMemcpyAsync(out, p.d_out, sizeof(double), hipMemcpyDeviceToHost, f->stream));
    HIPCHK(hipStreamSynchronize(f->stream));
    return SU3_OK;
}

int32_t su3_topological_charge(su3_field f, double* Q)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!Q) return fail(SU3_ERR_ARG, "Q is NULL");
    return scalar_reduction(f, 0, Q);
}

int32_t su3_clover_energy(su3_field f, double* E)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!E) return fail(SU3_ERR_ARG, "E is NULL");
    rc = scalar_reduction(f, 1, E);
    if (!rc) *E /= f->V;
    return rc;
}

// Class sums of Wilson loops (mode 0: all, 1: chi_munu, 2: chi), each class
// divided by its number of loops; extents are even, so a given pattern of odd
// coordinates holds exactly V / 16 sites.
static int32_t loop_classes(su3_field f, int m, int n, int mode, double* out)
{
    int32_t rc = single_plan(f, 5);
    if (rc) return rc;
    Plan& p = f->plan;
    const Grid g = p.grid_site();
    HIPCHK(launch_loops_partial(f->prec, g, m, n, mode, p.d_partials, f->stream));
    const int nclass = mode == 0 ? 1 : (mode == 1 ? 3 : 5);
    for (int c = 0; c < nclass; c++)
        HIPCHK(launch_reduce_final(g, p.d_partials + (size_t)c * p.nblk_site, p.d_out, 1, c, f->stream));
    double r[5];
    HIPCHK(hipMemcpyAsync(r, p.d_out, sizeof(double) * nclass, hipMemcpyDeviceToHost, f->stream));
    HIPCHK(hipStreamSynchronize(f->stream));
    static const double binom2[3] = { 1, 2, 1 }, binom4[5] = { 1, 4, 6, 4, 1 };
    for (int c = 0; c < nclass; c++) {
        double cnt;
        if (mode == 0)
            cnt = 6.0 * f->V;
        else if (mode == 1)
            cnt = 6.0 * binom2[c] * (f->V / 4.0);  // chi_munu sees the parities of 2 coordinates
        else
            cnt = 6.0 * binom4[c] * (f->V / 16.0);
        out[c] = r[c] / cnt;
    }
    return SU3_OK;
}

int32_t su3_wilson_loop(su3_field f, int32_t m, int32_t n, double* out)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!out) return fail(SU3_ERR_ARG, "out is NULL");
    if (m < 1 || n < 1 || m > 1024 || n > 1024) return fail(SU3_ERR_ARG, "loop extents must be in [1, 1024]");
    return loop_classes(f, m, n, 0, out);
}

int32_t su3_partial_plaquettes(su3_field f, double out[3])
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!out) return fail(SU3_ERR_ARG, "out is NULL");
    return loop_classes(f, 1, 1, 1, out);
}

int32_t su3_displaced_loops(su3_field f, double out[5])
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!out) return fail(SU3_ERR_ARG, "out is NULL");
    return loop_classes(f, 2, 2, 2, out);
}

int32_t su3_reunitarize(su3_field f)
{
    int32_t rc = check_field(f);
    if (!rc) rc = single_plan(f, 1);
    if (rc) return rc;
    HIPCHK(launch_reunit(f->prec, f->plan.grid_link(), f->plan.d_sweep, 0, 0, f->stream));
    return SU3_OK;
}

int32_t su3_gauge_transform(su3_field f, uint32_t seed)
{
    int32_t rc = check_field(f);
    if (!rc) rc = single_plan(f, 1);
    if (rc) return rc;
    HIPCHK(launch_gauge(f->prec, f->plan.grid_link(), seed, f->stream));
    return SU3_OK;
}

int32_t su3_check_field(su3_field f, double tol, double* max_dev, int64_t* worst)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    const int nb = ceil_div(8LL * f->Vh, 256);
    double* bm = nullptr;
    int* ba = nullptr;
    HIPCHK(hipMalloc(&bm, sizeof(double) * nb));
    if (hipMalloc(&ba, sizeof(int) * nb) != hipSuccess) {
        hipFree(bm);
        return fail(SU3_ERR_NOMEM, "check buffers");
    }
    std::vector<double> hm(nb);
    std::vector<int> ha(nb);
    hipError_t e = launch_check(f->prec, f->geo(), f->data, f->cs, bm, ba, nb, f->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hm.data(), bm, sizeof(double) * nb, hipMemcpyDeviceToHost, f->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ha.data(), ba, sizeof(int) * nb, hipMemcpyDeviceToHost, f->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    hipFree(bm);
    hipFree(ba);
    if (e != hipSuccess) return fail(SU3_ERR_HIP, std::string("check: ") + hipGetErrorString(e));
    double best = -1;
    int64_t arg = -1;
    for (int b = 0; b < nb; b++)
        if (hm[b] > best) {
            best = hm[b];
            arg = ha[b];
        }
    if (max_dev) *max_dev = best;
    if (worst) *worst = arg;
    if (!(best <= tol))
        return fail(SU3_ERR_NUMERIC, "link " + std::to_string(arg) + " deviates from SU(3) by " + std::to_string(best));
    return SU3_OK;
}

int32_t su3_hmc_trajectory(su3_field f, double beta, double tau, int32_t n_steps, uint32_t seed, uint32_t lattice_id,
                           uint64_t traj, int32_t metropolis, double* dH, int32_t* accepted)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (n_steps < 1) return fail(SU3_ERR_ARG, "n_steps must be >= 1");
    if (!std::isfinite(tau) || !std::isfinite(beta) || beta < 0) return fail(SU3_ERR_ARG, "tau and beta must be finite, beta >= 0");
    if ((rc = ensure_scratch(f, true, true))) return rc;
    if ((rc = single_plan(f, 4))) return rc;
    Plan& p = f->plan;
    hipStream_t st = f->stream;
    // descriptor variants: 0: U -> alt0, 1: alt0 -> alt1, 2: alt1 -> alt0
    std::vector<LatDesc> d(3, plan_desc(f));
    for (auto& x : d) {
        x.beta = beta;
        x.seed = seed;
        x.lid = lattice_id;
        x.aux = f->aux8;
    }
    d[0].U = f->data;
    d[0].aux2 = f->alt[0];
    d[1].U = f->alt[0];
    d[1].aux2 = f->alt[1];
    d[2].U = f->alt[1];
    d[2].aux2 = f->alt[0];
    HIPCHK(upload_descs(f->d_extra, d, st));
    const Grid g0 = p.grid_link(f->d_extra + 0);
    HIPCHK(launch_mom_refresh(f->prec, g0, traj, st));
    // H0
    double K0 = 0, S0 = 0;
    HIPCHK(launch_kinetic_partial(f->prec, g0, p.d_partials, st));
    HIPCHK(launch_reduce_final(g0, p.d_partials, p.d_out, 1, 0, st));
    HIPCHK(launch_plaq_partial(f->prec, p.grid_site(f->d_extra + 0), p.d_partials, st));
    HIPCHK(launch_reduce_final(p.grid_site(f->d_extra + 0), p.d_partials, p.d_out, 1, 1, st));
    const double eps = tau / n_steps;
    int cur = 0;  // descriptor whose U holds the current links
    for (int k = 0; k < n_steps; k++) {
        const double ek = (k == 0) ? 0.5 * eps : eps;
        HIPCHK(launch_kick_drift(f->prec, p.grid_lw(f->d_extra + cur), ek, eps, 1, st));
        cur = (cur == 1) ? 2 : 1;
    }
    HIPCHK(launch_kick_drift(f->prec, p.grid_lw(f->d_extra + cur), 0.5 * eps, 0.0, 0, st));
    HIPCHK(launch_kinetic_partial(f->prec, g0, p.d_partials, st));
    HIPCHK(launch_reduce_final(g0, p.d_partials, p.d_out, 1, 2, st));
    HIPCHK(launch_plaq_partial(f->prec, p.grid_site(f->d_extra + cur), p.d_partials, st));
    HIPCHK(launch_reduce_final(p.grid_site(f->d_extra + cur), p.d_partials, p.d_out, 1, 3, st));
    double r[4];
    HIPCHK(hipMemcpyAsync(r, p.d_out, sizeof r, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    K0 = r[0];
    S0 = beta * r[1];
    const double H0 = K0 + S0, H1 = r[2] + beta * r[3];
    const double dh = H1 - H0;
    int acc = 1;
    if (metropolis) {
        uint32_t c[4] = { 0u, (uint32_t)P_ACCEPT << 28, (uint32_t)traj, (uint32_t)(traj >> 32) };
        philox_host(c, seed, lattice_id);
        const double u = ((double)(c[0] >> 9) * 2.0 + 1.0) * 0x1p-24;
        acc = (u < std::exp(-dh)) ? 1 : 0;
    }
    if (acc) {
        void* src = (cur == 1) ? f->alt[0] : f->alt[1];
        HIPCHK(hipMemcpyAsync(f->data, src, f->bytes, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (dH) *dH = dh;
    if (accepted) *accepted = acc;
    return SU3_OK;
}

int32_t su3_wilson_flow(su3_field f, double eps, int32_t n_steps)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (n_steps < 0) return fail(SU3_ERR_ARG, "n_steps must be >= 0");
    if (!std::isfinite(eps)) return fail(SU3_ERR_ARG, "eps must be finite");
    if (n_steps == 0) return SU3_OK;
    if ((rc = ensure_scratch(f, true, true))) return rc;
    if ((rc = single_plan(f, 1))) return rc;
    hipStream_t st = f->stream;
    std::vector<LatDesc> d(2, plan_desc(f));
    d[0].U = f->data;
    d[0].aux2 = f->alt[0];
    d[1].U = f->alt[0];
    d[1].aux2 = f->data;
    for (auto& x : d) x.aux = f->aux8;
    HIPCHK(upload_descs(f->d_extra + 3, d, st));
    const double cz[3] = { 0.25, 8.0 / 9.0, 0.75 };
    const double ca[3] = { 0.0, -17.0 / 9.0, -1.0 };
    int cur = 0;
    for (int s = 0; s < n_steps; s++)
        for (int k = 0; k < 3; k++) {
            HIPCHK(launch_flow_stage(f->prec, f->plan.grid_lw(f->d_extra + 3 + cur), eps, cz[k], ca[k], k == 0, 0,
                                     nullptr, st));
            cur ^= 1;
        }
    if (cur == 1) HIPCHK(hipMemcpyAsync(f->data, f->alt[0], f->bytes, hipMemcpyDeviceToDevice, st));
    return SU3_OK;
}

// E (clover energy density) and Q of the links that descriptor d points at.
static int32_t measure_EQ(su3_field_s* f, const LatDesc* d, double* E, double* Q)
{
    Plan& p = f->plan;
    HIPCHK(launch_energy_partial(f->prec, p.grid_site(d), p.d_partials, f->stream));
    HIPCHK(launch_reduce_final(p.grid_site(d), p.d_partials, p.d_out, 1, 0, f->stream));
    HIPCHK(launch_qtop_partial(f->prec, p.grid_site(d), p.d_partials, f->stream));
    HIPCHK(launch_reduce_final(p.grid_site(d), p.d_partials, p.d_out, 1, 1, f->stream));
    double r[2];
    HIPCHK(hipMemcpyAsync(r, p.d_out, sizeof r, hipMemcpyDeviceToHost, f->stream));
    HIPCHK(hipStreamSynchronize(f->stream));
    *E = r[0] / f->V;
    *Q = r[1];
    return SU3_OK;
}

int32_t su3_wilson_flow_adaptive(su3_field f, double t_end, double tol, double max_step, double eps0,
                                 const double* t_meas, int32_t n_meas, double* E_out, double* Q_out,
                                 int32_t* n_accepted, int32_t* n_rejected)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!(t_end >= 0) || !std::isfinite(t_end)) return fail(SU3_ERR_ARG, "t_end must be finite and >= 0");
    if (!(tol > 0) || !(max_step > 0) || !(eps0 > 0) || !std::isfinite(max_step))
        return fail(SU3_ERR_ARG, "tol, max_step and eps0 must be positive");
    if (n_meas < 0 || (n_meas > 0 && (!t_meas || !E_out || !Q_out)))
        return fail(SU3_ERR_ARG, "measurement arrays are required for n_meas > 0");
    for (int k = 0; k < n_meas; k++)
        if (!std::isfinite(t_meas[k]) || t_meas[k] < 0 || t_meas[k] > t_end || (k > 0 && t_meas[k] <= t_meas[k - 1]))
            return fail(SU3_ERR_ARG, "measurement times must ascend within [0, t_end]");
    if ((rc = ensure_scratch(f, true, true, 3))) return rc;
    if ((rc = single_plan(f, 2))) return rc;
    Plan& p = f->plan;
    hipStream_t st = f->stream;
    // Buffers: W0 alternates between data (configuration 0) and alt0
    // (configuration 1); alt1 holds W2, alt2 the embedded W~.
    void* w0b[2] = { f->data, f->alt[0] };
    void* oth[2] = { f->alt[0], f->data };
    std::vector<LatDesc> d(6, plan_desc(f));
    for (int c = 0; c < 2; c++) {
        LatDesc* x = &d[3 * c];
        for (int k = 0; k < 3; k++) {
            x[k].aux = f->aux8;
            x[k].aux3 = f->alt[2];
            x[k].aux4 = w0b[c];
        }
        x[0].U = w0b[c];
        x[0].aux2 = oth[c];
        x[1].U = oth[c];
        x[1].aux2 = f->alt[1];
        x[2].U = f->alt[1];
        x[2].aux2 = oth[c];
    }
    HIPCHK(upload_descs(f->d_extra, d, st));
    const double cz[3] = { 0.25, 8.0 / 9.0, 0.75 };
    const double ca[3] = { 0.0, -17.0 / 9.0, -1.0 };
    int cfg = 0, k = 0, acc = 0, rej = 0;
    double t = 0, eps = std::min(eps0, max_step);
    while (k < n_meas && t_meas[k] <= 0) {
        if ((rc = measure_EQ(f, f->d_extra, &E_out[k], &Q_out[k]))) return rc;
        k++;
    }
    while (t < t_end) {
        const double target = (k < n_meas && t_meas[k] < t_end) ? t_meas[k] : t_end;
        const bool lands = eps >= target - t;
        const double h = lands ? target - t : eps;
        const Grid g0 = p.grid_lw(f->d_extra + 3 * cfg);
        for (int s = 0; s < 3; s++)
            HIPCHK(launch_flow_stage(f->prec, p.grid_lw(f->d_extra + 3 * cfg + s), h, cz[s], ca[s], s == 0, s,
                                     p.d_partials, st));
        HIPCHK(launch_reduce_max(g0, p.d_partials, p.d_out, st));
        double dist = 0;
        HIPCHK(hipMemcpyAsync(&dist, p.d_out, sizeof dist, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (!std::isfinite(dist)) return fail(SU3_ERR_NUMERIC, "adaptive flow: non-finite error estimate");
        if (dist <= tol) {
            acc++;
            cfg ^= 1;  // W3 sits in the other buffer, which now holds W0
            t = lands ? target : t + h;
            while (k < n_meas && t_meas[k] <= t) {
                if ((rc = measure_EQ(f, f->d_extra + 3 * cfg, &E_out[k], &Q_out[k]))) return rc;
                k++;
            }
        } else {
            rej++;
        }
        eps = dist > 0 ? std::min(max_step, 0.95 * h * std::cbrt(tol / dist)) : max_step;
        if (rej > 100000 || !(eps > 1e-12)) return fail(SU3_ERR_NUMERIC, "adaptive flow: step size collapsed");
    }
    if (cfg == 1) HIPCHK(hipMemcpyAsync(f->data, f->alt[0], f->bytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    if (n_accepted) *n_accepted = acc;
    if (n_rejected) *n_rejected = rej;
    return SU3_OK;
}

int32_t su3_max_plaquette_action(su3_field f, double* h)
{
    int32_t rc = check_field(f);
    if (rc) return rc;
    if (!h) return fail(SU3_ERR_ARG, "h is NULL");
    if ((rc = single_plan(f, 1))) return rc;
    Plan& p = f->plan;
    HIPCHK(launch_max_splaq_partial(f->prec, p.grid_site(), p.d_partials, f->stream));
    HIPCHK(launch_reduce_max(p.grid_site(), p.d_partials, p.d_out, f->stream));
    HIPCHK(hipMemcpyAsync(h, p.d_out, sizeof(double), hipMemcpyDeviceToHost, f->stream));
    HIPCHK(hipStreamSynchronize(f->stream));
    return SU3_OK;
}

int32_t su3_flow_t0(const double* t, const double* E, int32_t n, double target, double* t0)
{
    if (!t || !E || !t0 || n < 2) return fail(SU3_ERR_ARG, "need t, E (n >= 2) and t0");
    for (int k = 1; k < n; k++) {
        const double y0 = t[k - 1] * t[k - 1] * E[k - 1], y1 = t[k] * t[k] * E[k];
        if (y0 < target && y1 >= target) {
            *t0 = t[k - 1] + (target - y0) * (t[k] - t[k - 1]) / (y1 - y0);
            return SU3_OK;
        }
    }
    return fail(SU3_ERR_NUMERIC, "t^2 E(t) does not cross the target between the given times");
}

int32_t su3_restrict(su3_field fine, su3_field coarse)
{
    int32_t rc = check_field(fine);
    if (!rc) rc = check_field(coarse);
    if (rc) return rc;
    for (int m = 0; m < 4; m++)
        if (fine->L[m] != 2 * coarse->L[m]) return fail(SU3_ERR_SHAPE, "fine dims must be twice the coarse dims");
    if (fine->stream != coarse->stream) HIPCHK(hipStreamSynchronize(fine->stream));
    HIPCHK(launch_restrict(fine->prec, fine->geo(), fine->data, fine->cs, coarse->prec, coarse->geo(), coarse->data,
                           coarse->cs, coarse->stream));
    return SU3_OK;
}

int32_t su3_prolongate(su3_field coarse, su3_field fine, double c, double rel_tol, int32_t max_iter,
                       int32_t iters_out[3])
{
    int32_t rc = check_field(fine);
    if (!rc) rc = check_field(coarse);
    if (rc) return rc;
    for (int m = 0; m < 4; m++)
        if (fine->L[m] != 2 * coarse->L[m]) return fail(SU3_ERR_SHAPE, "fine dims must be twice the coarse dims");
    if (!(c > 0) || !std::isfinite(c)) return fail(SU3_ERR_ARG, "c must be > 0");
    if (!(rel_tol >= 0)) return fail(SU3_ERR_ARG, "rel_tol must be >= 0");
    if (max_iter < 0) return fail(SU3_ERR_ARG, "max_iter must be >= 0");
    hipStream_t st = fine->stream;
    if (coarse->stream != st) HIPCHK(hipStreamSynchronize(coarse->stream));
    const Geo gf = fine->geo();
    const size_t csf = slab_bytes(fine->Vh, 18, 8);
    const size_t nbytes = 8 * csf;
    double* buf[2] = { nullptr, nullptr };
    const int nb = std::max({ ape_blocks(gf, 0), ape_blocks(gf, 1), ape_blocks(gf, 2) });
    double* bs = nullptr;
    void* state = nullptr;
    if (hipMalloc(&buf[0], nbytes) != hipSuccess || hipMalloc(&buf[1], nbytes) != hipSuccess ||
        hipMalloc(&bs, sizeof(double) * nb) != hipSuccess || hipMalloc(&state, ape_state_bytes()) != hipSuccess) {
        hipFree(buf[0]);
        hipFree(buf[1]);
        hipFree(bs);
        hipFree(state);
        return fail(SU3_ERR_NOMEM, "prolongation scratch allocation failed");
    }
    hipError_t e = launch_transfer(coarse->prec, coarse->geo(), coarse->data, coarse->cs, gf, buf[0], csf, st);
    int cur = 0;
    int iters[3] = { 0, 0, 0 };
    // Steps are enqueued in runs of `run` without waiting; the stage's state
    // on the device turns the steps after the stopping point into no-ops.
    const int run = 16;
    for (int d = 0; d < 3 && e == hipSuccess; d++) {
        // a step writes only the bonds of stage d: both buffers start the
        // stage with the same links
        e = hipMemcpyAsync(buf[cur ^ 1], buf[cur], nbytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = launch_ape_reset(state, st);
        const int nbd = ape_blocks(gf, d);
        int done = max_iter == 0, k = 0;
        for (int j = 1; e == hipSuccess && !done; j++) {
            // step j reads iterate j-1 from buf[cur ^ ((j-1) & 1)]
            const int src = cur ^ ((j - 1) & 1);
            e = launch_ape_step(gf, buf[src], buf[src ^ 1], csf, d, c, j, rel_tol, max_iter, state, bs, nbd, st);
            if (e == hipSuccess && (j % run == 0 || j >= max_iter)) e = read_ape_state(state, &done, &k, st);
        }
        iters[d] = k;
        cur ^= k & 1;
    }
    if (e == hipSuccess) e = launch_convert(fine->prec, fine->data, fine->cs, PREC_F64, buf[cur], csf, fine->Vh, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(buf[0]);
    hipFree(buf[1]);
    hipFree(bs);
    hipFree(state);
    if (e != hipSuccess) return fail(SU3_ERR_HIP, std::string("prolongate: ") + hipGetErrorString(e));
    if (iters_out)
        for (int d = 0; d < 3; d++) iters_out[d] = iters[d];
    return SU3_OK;
}

int32_t su3_set_launch(int32_t block, int32_t xcd_remap)
{
    if (!(block == 0 || block == 64 || block == 128 || block == 256 || block == 512))
        return fail(SU3_ERR_ARG, "block must be 0, 64, 128, 256 or 512");
    if (xcd_remap != 0 && xcd_remap != 1) return fail(SU3_ERR_ARG, "xcd_remap must be 0 or 1");
    std::lock_guard<std::mutex> lk(g_mu);
    g_forced_block = block;
    g_forced_remap = xcd_remap;
    return SU3_OK;
}

int32_t su3_set_group_bytes(uint64_t bytes)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_group_bytes = (size_t)bytes;
    return SU3_OK;
}

int32_t su3_set_tile(int32_t ty, int32_t tz, int32_t tt)
{
    if (ty < 0 || tz < 0 || tt < 0) return fail(SU3_ERR_ARG, "tile extents must be >= 0");
    std::lock_guard<std::mutex> lk(g_mu);
    g_tile_forced = !(ty == 0 && tz == 0 && tt == 0);
    g_forced_tile[0] = ty;
    g_forced_tile[1] = tz;
    g_forced_tile[2] = tt;
    return SU3_OK;
}

int32_t su3_get_config(const su3_field* fs, int32_t n, int32_t out[5])
{
    if (!fs || n <= 0 || !out) return fail(SU3_ERR_ARG, "need fields and an output array");
    std::vector<su3_field_s*> v;
    for (int i = 0; i < n; i++) {
        if (!fs[i]) return fail(SU3_ERR_ARG, "NULL field");
        v.push_back(fs[i]);
    }
    const LaunchCfg c = launch_choice(v);
    out[0] = c.block;
    out[1] = c.remap;
    out[2] = c.ty;
    out[3] = c.tz;
    out[4] = c.tt;
    return SU3_OK;
}

int32_t su3_get_launch(int32_t* block, int32_t* xcd_remap)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (block) *block = g_forced_block;
    if (xcd_remap) *xcd_remap = g_forced_remap;
    return SU3_OK;
}

int32_t su3_autotune(int32_t enable)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_autotune = enable != 0;
    return SU3_OK;
}

int32_t su3_profile_enable(int32_t enable)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_profile = enable != 0;
    g_prof_ms[0] = g_prof_ms[1] = g_prof_ms[2] = 0;
    g_prof_n[0] = g_prof_n[1] = g_prof_n[2] = 0;
    return SU3_OK;
}

int32_t su3_profile_read(int32_t kind, double* total_ms, int64_t* launches)
{
    if (kind < 0 || kind > 2) return fail(SU3_ERR_ARG, "kind must be 0, 1 or 2");
    std::lock_guard<std::mutex> lk(g_mu);
    if (total_ms) *total_ms = g_prof_ms[kind];
    if (launches) *launches = g_prof_n[kind];
    return SU3_OK;
}

}  // extern "C"
