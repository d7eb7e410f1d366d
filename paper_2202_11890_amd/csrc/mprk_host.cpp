// mprk_host.cpp -- host side of the MPRK library: configuration checks,
// workspace layout, the stage schedule of one slow step (Algorithm 1 in a
// low-storage substep form), execution modes (one launch per stage, a graph
// per slow step, one persistent launch per run segment), batches of
// independent members, the tile-shape autotuner and the device reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mprk.h"
#include "mprk_internal.h"

using namespace mprk;

namespace {

constexpr size_t ALIGN = 256;

size_t round_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

void set_msg(char* msg, size_t len, const char* fmt, ...)
{
    if (!msg || len == 0) return;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, len, fmt, ap);
    va_end(ap);
}

// Base methods in Shu-Osher form: stage j (1-based) computes
// Q_{j+1} = alpha_j U + (1 - alpha_j)(Q_j + h R(Q_j)), Q_1 = U; the last stage
// gives U + h sum_j b_j R_j.
//   2 stages (the RK2 base of Table 1, A21 = 1, b = (1/2, 1/2)): alpha = 0, 1/2.
//   3 stages (SSP-RK3, A21 = 1, A31 = A32 = 1/4, b = (1/6, 1/6, 2/3)):
//     alpha = 0, 3/4, 1/3.
int shu_osher(int base, double* alpha)
{
    if (base == 2) { alpha[0] = 0.0; alpha[1] = 0.5; return 2; }
    if (base == 3) { alpha[0] = 0.0; alpha[1] = 0.75; alpha[2] = 1.0 / 3.0; return 3; }
    return -1;
}

int tiles_of(int n, int t) { return (n + t - 1) / t; }

// Default 2D tile shape (measured on the 1024x512 workload: 32x16 is the
// fastest with FP64 and with FP32 fluxes).  3D contexts ignore the 2D shape.
int default_shape(const mprk_config&)
{
    return TILE_32x16;
}

int nv_of(const mprk_config& c) { return c.dim == 3 ? NV3 : NV; }

// Fixed tiles of both domains for a tile shape (3D: the 3D kernel's tile).
int member_tiles(const mprk_config& c, int shape)
{
    if (c.dim == 3) {
        const TileDims3 d = tile3_dims(c.flux_bits == 32);
        return tiles_of(c.nx, d.tx) * tiles_of(c.ny, d.ty) *
               (tiles_of(c.nz_lower, d.tz) + tiles_of(c.nz_upper, d.tz));
    }
    const TileDims d = tile_dims(shape);
    return tiles_of(c.nx, d.tx) * (tiles_of(c.nz_lower, d.tz) + tiles_of(c.nz_upper, d.tz));
}

int max_member_tiles(const mprk_config& c)
{
    int n = 0;
    for (int sh = 0; sh < TILE_SHAPES; ++sh) n = std::max(n, member_tiles(c, sh));
    return n;
}

// Per-member device scratch: stage arrays, retained slow rows, the buffer
// accumulator and the reduction partials.
struct CoreLayout {
    int s;
    size_t n_lo, n_up;        // doubles per state array
    size_t off_stage_lo[3];   // stage arrays Q_2..Q_s of each domain
    size_t off_stage_up[3];
    size_t off_ret[3];        // retained slow rows per base stage
    size_t off_acc;
    size_t off_partial, off_final;
    size_t total;
};

bool core_layout(const mprk_config* c, CoreLayout* L)
{
    double al[3];
    int s = shu_osher(c->base_rk, al);
    if (s < 0) return false;
    L->s = s;
    const size_t nv = nv_of(*c), row = (size_t)c->nx * (c->dim == 3 ? c->ny : 1);
    L->n_lo = nv * c->nz_lower * row;
    L->n_up = nv * c->nz_upper * row;
    size_t off = 0;
    for (int j = 0; j < 3; ++j) { L->off_stage_lo[j] = L->off_stage_up[j] = 0; L->off_ret[j] = 0; }
    for (int j = 0; j < s - 1; ++j) {
        L->off_stage_lo[j] = off;
        off += round_up(L->n_lo * sizeof(double));
        L->off_stage_up[j] = off;
        off += round_up(L->n_up * sizeof(double));
    }
    const bool multi = c->m > 1;
    for (int j = 0; j < s; ++j) {
        L->off_ret[j] = off;
        if (multi) off += round_up(nv * 2 * row * sizeof(double));
    }
    L->off_acc = off;
    if (multi) off += round_up(nv * c->n_buffer * row * sizeof(double));
    L->off_partial = off;
    off += round_up((size_t)2 * RED_BLOCKS * RED_FIELDS * sizeof(double));
    L->off_final = off;
    off += round_up((size_t)2 * RED_FIELDS * sizeof(double));
    L->total = off;
    return true;
}

// A context's tables after its core scratch: persistent execution (stage
// records, tile list, member record, progress counters + abort flag).
struct CtxLayout {
    CoreLayout core;
    size_t off_ptab, off_ptiles, off_pmember, off_pdone;
    int max_tiles;
    size_t total;
};

bool ctx_layout(const mprk_config* c, CtxLayout* L)
{
    if (!core_layout(c, &L->core)) return false;
    size_t off = L->core.total;
    L->max_tiles = max_member_tiles(*c);
    L->off_ptab = off;
    off += round_up((size_t)c->m * L->core.s * sizeof(StageArgs));
    L->off_ptiles = off;
    off += round_up((size_t)L->max_tiles * sizeof(TileRef));
    L->off_pmember = off;
    off += round_up(sizeof(MemberRun));
    L->off_pdone = off;
    off += round_up((size_t)(L->max_tiles + 1) * sizeof(int32_t));
    L->total = off;
    return true;
}

// One coupled two-domain problem bound to its state and scratch: what the
// stage schedule needs.
struct Member {
    mprk_config cfg;
    CoreLayout lay;
    double* q[2];           // lower, upper (caller-owned device memory)
    char* ws;               // this member's scratch (device)
    double alpha[3];
    int fast, slow;         // domain indices
    int b_lo, b_hi, ret_lo; // buffer rows and retained rows of the slow domain

    void init(const mprk_config& g, const CoreLayout& L, double* ql, double* qu, char* w)
    {
        cfg = g;
        lay = L;
        q[0] = ql;
        q[1] = qu;
        ws = w;
        shu_osher(g.base_rk, alpha);
        fast = g.fast_is_lower ? 0 : 1;
        slow = 1 - fast;
        const int nzs = g.fast_is_lower ? g.nz_upper : g.nz_lower;
        if (g.fast_is_lower) {
            b_lo = 0;
            b_hi = g.n_buffer;
            ret_lo = g.n_buffer;
        } else {
            b_lo = nzs - g.n_buffer;
            b_hi = nzs;
            ret_lo = b_lo - 2;
        }
    }
    double* stage(int dom, int j) const   // Q_{j+1}, j = 1..s-1
    {
        return (double*)(ws + (dom == 0 ? lay.off_stage_lo[j - 1] : lay.off_stage_up[j - 1]));
    }
    double* ret(int j) const { return (double*)(ws + lay.off_ret[j]); }
    double* acc() const { return (double*)(ws + lay.off_acc); }
    int ms() const { return cfg.m * lay.s; }
};

// Shared per-launch constants; domain-specific fields are filled by callers.
StageArgs base_args(const Member& mb)
{
    const mprk_config& g = mb.cfg;
    StageArgs a;
    std::memset(&a, 0, sizeof a);
    a.nx = g.nx;
    a.ny = g.dim == 3 ? g.ny : 1;
    a.dy = g.dim == 3 ? g.dy : 0.0;
    a.inv_dy = g.dim == 3 ? 1.0 / g.dy : 0.0;
    a.dx = g.dx;
    a.inv_dx = 1.0 / g.dx;
    a.hinv_dx = 0.5 * a.inv_dx;
    a.hinv_dy = 0.5 * a.inv_dy;
    a.gamma = g.gamma;
    a.gm1 = g.gamma - 1.0;
    a.inv_dx_f = (float)a.inv_dx;
    a.inv_dy_f = (float)a.inv_dy;
    a.gamma_f = (float)a.gamma;
    a.gm1_f = (float)a.gm1;
    a.gravity = g.gravity;
    const double mu1 = g.mu_lower, mu2 = g.mu_upper;
    const double k1 = mu1 / ((g.gamma - 1.0) * g.prandtl);
    const double k2 = mu2 / ((g.gamma - 1.0) * g.prandtl);
    const double dz1 = g.dz_lower, dz2 = g.dz_upper;
    a.bu = 2.0 * mu1 * mu2 / (dz2 * mu1 + dz1 * mu2);
    a.bT = 2.0 * k1 * k2 / (dz2 * k1 + dz1 * k2);
    a.half_dz1_mu1 = dz1 / (2.0 * mu1);
    a.inv_m = 1.0 / g.m;
    a.flux32 = g.flux_bits == 32 ? 1 : 0;
    for (int d = 0; d < 2; ++d) {
        DomainArgs& D = a.d[d];
        D.nz = d == 0 ? g.nz_lower : g.nz_upper;
        D.dz = d == 0 ? dz1 : dz2;
        D.inv_dz = 1.0 / D.dz;
        D.hinv_dz = 0.5 * D.inv_dz;
        D.mu = d == 0 ? mu1 : mu2;
        D.kappa = d == 0 ? k1 : k2;
        D.inv_dz_f = (float)D.inv_dz;
        D.mu_f = (float)D.mu;
        D.kappa_f = (float)D.kappa;
        // Viscous coefficients per direction (x, y, z), folded so that a face
        // scales raw differences of the staged primitives once.
        const double inv_h[3] = {a.inv_dx, a.inv_dy, D.inv_dz};
        for (int k = 0; k < 3; ++k) {
            D.vk[VK_NN][k] = (4.0 / 3.0) * D.mu * inv_h[k];
            D.vk[VK_N][k] = D.mu * inv_h[k];
            D.vk[VK_Q][k] = 2.0 * D.kappa * inv_h[k];
            D.vk[VK_TT][k] = (-2.0 / 3.0) * D.mu * (0.25 * inv_h[k]);
            D.vk[VK_TN][k] = D.mu * (0.25 * inv_h[k]);
            for (int r = 0; r < 5; ++r) D.vk_f[r][k] = (float)D.vk[r][k];
        }
        D.gamma_top = d == 0;
        D.gamma_bot = d == 1;
        D.b_lo = D.b_hi = 0;
        D.ret_lo = 0;
    }
    return a;
}

// Tiles of a launch over rows (z-planes) [lo, hi): fixed tiles, z aligned at
// multiples of the tile height.  shape < 0 selects the 3D kernel's tile.
void set_rows(DomainArgs& D, const mprk_config& g, int lo, int hi, int shape)
{
    int tx, ty = 1, tz;
    if (g.dim == 3) {
        const TileDims3 t = tile3_dims(g.flux_bits == 32);
        tx = t.tx;
        ty = t.ty;
        tz = t.tz;
    } else {
        const TileDims t = tile_dims(shape);
        tx = t.tx;
        tz = t.tz;
    }
    D.row_lo = lo;
    D.row_hi = hi;
    D.tiles_x = tiles_of(g.nx, tx);
    D.tiles_y = g.dim == 3 ? tiles_of(g.ny, ty) : 1;
    D.tiles_z = hi > lo ? (hi - 1) / tz - lo / tz + 1 : 0;   // fixed tiles meeting [lo, hi)
    D.ntiles = D.tiles_x * D.tiles_y * D.tiles_z;
}

// Block count and block order of a stage record: launches that cover only
// the buffer band of the slow domain put its (short) tiles first, so they run
// in the first wave of workgroups.
void finish_record(const Member& mb, StageArgs& a)
{
    a.nblocks = a.d[0].ntiles + a.d[1].ntiles;
    a.first = a.d[mb.slow].use_ret ? mb.slow : 0;
}

Combine combine(double alpha, double h, int mode)
{
    Combine cb;
    cb.alpha = alpha;
    cb.beta = 1.0 - alpha;
    cb.bh = (1.0 - alpha) * h;
    cb.mode = mode;
    cb.pad = 0;
    return cb;
}

// Launch parameters of global stage (k, j) of a slow step of size dt
// (Algorithm 1 in the low-storage substep form).
StageArgs stage_args(const Member& mb, double dt, int k, int j, int shape)
{
    const mprk_config& g = mb.cfg;
    const int s = mb.lay.s, m = g.m;
    const int F = mb.fast, S = mb.slow;
    double* qF = mb.q[F];
    double* qS = mb.q[S];
    const int nzF = F == 0 ? g.nz_lower : g.nz_upper;
    const int nzS = S == 0 ? g.nz_lower : g.nz_upper;
    const double hF = dt / m;
    StageArgs a = base_args(mb);
    const double al = mb.alpha[j - 1];
    const bool last = (j == s);

    // Fast domain: m substeps of dt/m of the base method.
    DomainArgs& DF = a.d[F];
    DF.qin = (j == 1) ? qF : mb.stage(F, j - 1);
    DF.base = qF;
    DF.out = last ? qF : mb.stage(F, j);
    DF.main = combine(al, hF, MODE_STAGE);
    DF.buf = DF.main;
    set_rows(DF, g, 0, nzF, shape);

    // Slow domain.
    DomainArgs& DS = a.d[S];
    DS.qin = (j == 1) ? qS : mb.stage(S, j - 1);
    DS.base = qS;
    DS.out = last ? qS : mb.stage(S, j);
    if (m == 1) {
        // Single rate: buffer and slow rows are the same base step.
        DS.main = combine(al, dt, MODE_STAGE);
        DS.buf = DS.main;
        set_rows(DS, g, 0, nzS, shape);
    } else {
        DS.b_lo = mb.b_lo;
        DS.b_hi = mb.b_hi;
        DS.ret_lo = mb.ret_lo;
        DS.acc = mb.acc();
        // Buffer: each substep restarts from q^B_n with the full step; the
        // results of the m trial steps are averaged.
        int bmode = MODE_STAGE;
        if (last) bmode = (k == 1) ? MODE_ACC_FIRST : (k < m ? MODE_ACC_ADD : MODE_ACC_FINAL);
        DS.buf = combine(al, dt, bmode);
        DS.main = combine(al, dt, MODE_STAGE);
        if (k == 1) {
            // Slow rows: one base step; keep the two rows next to the buffer of
            // each stage value for the later substeps.
            DS.ret_out = mb.ret(j - 1);
            set_rows(DS, g, 0, nzS, shape);
        } else {
            DS.use_ret = 1;
            DS.ret_in = mb.ret(j - 1);
            set_rows(DS, g, mb.b_lo, mb.b_hi, shape);
        }
    }
    finish_record(mb, a);
    return a;
}

// The same rows and tiles as stage (k, j) but writing R(state) into the
// stage scratch and leaving the state alone: the workload the autotuner
// times.
StageArgs proxy_args(const Member& mb, double dt, int k, int j, int shape)
{
    StageArgs a = stage_args(mb, dt, k, j, shape);
    for (int d = 0; d < 2; ++d) {
        DomainArgs& D = a.d[d];
        D.qin = mb.q[d];
        D.base = mb.q[d];
        D.out = mb.stage(d, 1);
        D.acc = nullptr;
        D.ret_in = nullptr;
        D.ret_out = nullptr;
        D.use_ret = 0;
        D.main = combine(0.0, 0.0, MODE_RHS);
        D.buf = D.main;
    }
    finish_record(mb, a);
    return a;
}

// Reduction record of a state pair (partials and finals where given).
ReduceArgs reduce_args(const mprk_config& g, const double* q_lower, const double* q_upper,
                       double* partial, double* final_)
{
    ReduceArgs r;
    std::memset(&r, 0, sizeof r);
    r.q[0] = q_lower;
    r.q[1] = q_upper;
    r.nz[0] = g.nz_lower;
    r.nz[1] = g.nz_upper;
    r.nx = g.nx;
    r.ny = g.dim == 3 ? g.ny : 1;
    r.nv = nv_of(g);
    r.inv_dx = 1.0 / g.dx;
    r.inv_dy = g.dim == 3 ? 1.0 / g.dy : 0.0;
    r.inv_dz[0] = 1.0 / g.dz_lower;
    r.inv_dz[1] = 1.0 / g.dz_upper;
    const double coef = std::max(4.0 / 3.0, g.gamma / g.prandtl);
    const double hy = g.dim == 3 ? 1.0 / (g.dy * g.dy) : 0.0;
    r.visc_coef[0] = coef * g.mu_lower * (1.0 / (g.dx * g.dx) + hy + 1.0 / (g.dz_lower * g.dz_lower));
    r.visc_coef[1] = coef * g.mu_upper * (1.0 / (g.dx * g.dx) + hy + 1.0 / (g.dz_upper * g.dz_upper));
    r.gamma = g.gamma;
    r.gm1 = g.gamma - 1.0;
    r.partial = partial;
    r.final_ = final_;
    return r;
}

// Reduction record of one member (partials in its scratch; finals at final_).
ReduceArgs member_reduce_args(const Member& mb, double* final_)
{
    return reduce_args(mb.cfg, mb.q[0], mb.q[1], (double*)(mb.ws + mb.lay.off_partial), final_);
}

// Device reductions of one member: totals, stability measures, status.
int member_reduce_launch(const Member& mb, hipStream_t stream, double* host_final)
{
    const ReduceArgs r = member_reduce_args(mb, (double*)(mb.ws + mb.lay.off_final));
    if (launch_reduce(r, stream) != hipSuccess) return MPRK_EHIP;
    if (hipMemcpyAsync(host_final, r.final_, 2 * RED_FIELDS * sizeof(double), hipMemcpyDeviceToHost,
                       stream) != hipSuccess)
        return MPRK_EHIP;
    return MPRK_OK;
}

// Stats from the reduced fields (after the stream is synchronised).
int stats_from_final(const mprk_config& g, const double* host_final, int64_t steps, mprk_stats* out)
{
    mprk_stats st;
    std::memset(&st, 0, sizeof st);
    const double dy = g.dim == 3 ? g.dy : 1.0;
    const double cellv[2] = {g.dx * dy * g.dz_lower, g.dx * dy * g.dz_upper};
    const int nv = nv_of(g);
    int bad = 0;
    for (int d = 0; d < 2; ++d) {
        const double* f = host_final + d * RED_FIELDS;
        double* tot = d == 0 ? st.totals_lower : st.totals_upper;
        for (int v = 0; v < nv; ++v) tot[v] = (f[v] + f[5 + v]) * cellv[d];
        (d == 0 ? st.lambda_lower : st.lambda_upper) = f[10];
        (d == 0 ? st.courant_lower : st.courant_upper) = f[11];
        (d == 0 ? st.visc_lower : st.visc_upper) = f[12];
        if (f[13] != 0.0) bad = 1;
    }
    st.steps_done = steps;
    st.status = bad;
    if (out) *out = st;
    return bad ? MPRK_ENONFINITE : MPRK_OK;
}

int member_stats(const Member& mb, const double* host_final, int64_t steps, mprk_stats* out)
{
    return stats_from_final(mb.cfg, host_final, steps, out);
}

// Device properties needed by the persistent mode.
int persistent_setup(bool flux32, int shape, int ntiles, double wait_seconds, int* grid,
                     int64_t* wait_ticks)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MPRK_EHIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MPRK_EHIP;
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop)
        return MPRK_EUNSUPPORTED;
    const int per_cu = persistent_blocks_per_cu(flux32, shape);
    if (per_cu <= 0) return MPRK_EHIP;
    int gsz = per_cu * prop.multiProcessorCount;
    if (gsz > ntiles) gsz = ntiles;
    *grid = gsz;
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        rate_khz <= 0)
        rate_khz = 100000;
    *wait_ticks = (int64_t)((double)rate_khz * 1000.0 * wait_seconds);
    return MPRK_OK;
}

// Tile list and member record of one member for persistent execution.
void persistent_member(const Member& mb, int member, int shape, int done_base,
                       std::vector<TileRef>& tiles, MemberRun& mr)
{
    const TileDims t = tile_dims(shape);
    const mprk_config& g = mb.cfg;
    const int tx = tiles_of(g.nx, t.tx);
    const int tz[2] = {tiles_of(g.nz_lower, t.tz), tiles_of(g.nz_upper, t.tz)};
    for (int d = 0; d < 2; ++d)
        for (int z = 0; z < tz[d]; ++z)
            for (int x = 0; x < tx; ++x) tiles.push_back(TileRef{member, d, x, z});
    std::memset(&mr, 0, sizeof mr);
    mr.tiles_x = tx;
    mr.tiles_z[0] = tz[0];
    mr.tiles_z[1] = tz[1];
    mr.done_base[0] = done_base;
    mr.done_base[1] = done_base + tx * tz[0];
}

// A graph of kernel nodes executed in order (one slow step).
struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void reset()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    bool begin()
    {
        reset();
        return hipGraphCreate(&graph, 0) == hipSuccess;
    }
    // Appends a kernel node after the previous one.
    bool add(const KernelRef& k, int blocks, void** args, hipGraphNode_t* prev)
    {
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof p);
        p.func = (void*)k.func;
        p.gridDim = dim3(blocks);
        p.blockDim = dim3(k.block);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node;
        if (hipGraphAddKernelNode(&node, graph, *prev ? prev : nullptr, *prev ? 1 : 0, &p) != hipSuccess)
            return false;
        *prev = node;
        return true;
    }
    bool finish() { return hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess; }
};

bool valid_mode(int mode)
{
    return mode == MPRK_EXEC_LAUNCH || mode == MPRK_EXEC_PERSISTENT || mode == MPRK_EXEC_GRAPH;
}

}  // namespace

struct mprk_ctx {
    CtxLayout lay;
    Member mb;
    hipStream_t stream;
    int64_t steps = 0;
    double host_final[2 * RED_FIELDS];
    int exec = MPRK_EXEC_LAUNCH;
    int shape = TILE_32x16;
    // persistent execution
    double ptab_dt = 0.0;                     // dt of the uploaded stage table (0: none)
    int ptab_shape = -1;
    int ptiles_shape = -1;
    int pgrid = 0;                            // persistent grid size (0: recompute)
    int64_t wait_ticks = 0;
    double wait_seconds = 10.0;
    std::vector<StageArgs> h_tab;             // host copies read by the async uploads
    std::vector<TileRef> h_tiles;
    MemberRun h_mr;
    // graph execution: one slow step
    StepGraph graph;
    std::vector<StageArgs> g_args;            // argument blocks the graph nodes point to
    std::vector<void*> g_ptrs;
    double graph_dt = 0.0;
    int graph_shape = -1;
    // kernel timing
    bool prof_on = false;
    size_t prof_used = 0;                     // event pairs recorded since the last take
    std::vector<hipEvent_t> prof_ev;          // start/stop pairs, reused
};

struct mprk_batch {
    int n = 0;
    std::vector<Member> mb;
    std::vector<double> dt;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    bool flux32 = false;
    int exec = MPRK_EXEC_LAUNCH;
    int shape = TILE_32x16;
    int64_t steps = 0;
    int nslots = 0;                           // launches per slow step (max m*s)
    int total_ms = 0;                         // stage records per slow step, all members
    std::vector<int> rec0;                    // first stage record of each member
    std::vector<int> slot_stage;              // [member][slot]: stage record or -1
    // device tables (offsets into ws)
    size_t off_tab, off_proxy, off_bmap, off_slots, off_ptiles, off_pmember, off_pdone;
    size_t off_red, off_finals;
    bool red_ready = false;
    std::vector<ReduceArgs> h_red;
    int max_tiles = 0;
    // host tables for the current shape
    int tab_shape = -1;
    bool rec_dirty = false;                   // steps changed: stage records to rewrite
    int rec_dev = 0;                          // dev_stores of the records on the device
    std::vector<StageArgs> h_tab, h_proxy;
    std::vector<BatchEntry> h_bmap;           // [slot][block] (first slot_blocks entries used)
    std::vector<int> slot_count, slot_blocks;
    std::vector<TileRef> h_tiles;
    std::vector<MemberRun> h_mr;
    std::vector<int32_t> h_slots;
    int pgrid = 0, pgrid_shape = -1;
    int64_t wait_ticks = 0;
    double wait_seconds = 10.0;
    StepGraph graph;
    int graph_shape = -1;
    std::vector<std::vector<void*>> g_args;   // per node: pointers to its argument values
    struct NodeArgs { const StageArgs* tab; const BatchEntry* bmap; int nblocks; };
    std::vector<NodeArgs> g_vals;
    std::vector<double> host_final;           // [member][2*RED_FIELDS]
    double adapt_cr = 0.0, adapt_dn = 0.0;    // adaptive steps at check points (cr 0: off)
    std::vector<mprk_stats> chk;              // stats of the last check
};

namespace {

// ---- single context ------------------------------------------------------

// Result-store policy of a 2D problem (see st_dev): device-scope stores from
// 2^17 cells (both domains) up.  Measured per step on single contexts: 5-7%
// faster from 512x256 per domain up, 1-2% slower at 256x128 and below, where
// a launch's output stays in the L2 for the next one.
bool big_2d(const mprk_config& g)
{
    return g.dim == 2 && (int64_t)g.nx * (g.nz_lower + g.nz_upper) >= (1 << 17);
}

// Stage records of a single context: the policy above (3D keeps ordinary
// stores, which measured faster there).
StageArgs ctx_stage_args(const mprk_ctx* c, double dt, int k, int j)
{
    StageArgs a = stage_args(c->mb, dt, k, j, c->shape);
    a.dev_stores = big_2d(c->mb.cfg) ? 1 : 0;
    return a;
}

hipError_t launch_any(const mprk_ctx* c, const StageArgs& a)
{
    if (c->mb.cfg.dim == 3) return launch_stage3(a, c->stream);
    return launch_stage(a, c->shape, c->stream);
}

hipError_t launch_any(const mprk_ctx* c, const StageArgs& a);

int launch(mprk_ctx* c, const StageArgs& a)
{
    if (!c->prof_on) return launch_any(c, a) == hipSuccess ? MPRK_OK : MPRK_EHIP;
    if (2 * c->prof_used + 2 > c->prof_ev.size()) {
        for (int i = 0; i < 2; ++i) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) return MPRK_EHIP;
            c->prof_ev.push_back(ev);
        }
    }
    hipEvent_t e0 = c->prof_ev[2 * c->prof_used], e1 = c->prof_ev[2 * c->prof_used + 1];
    if (hipEventRecord(e0, c->stream) != hipSuccess) return MPRK_EHIP;
    if (launch_any(c, a) != hipSuccess) return MPRK_EHIP;
    if (hipEventRecord(e1, c->stream) != hipSuccess) return MPRK_EHIP;
    c->prof_used += 1;
    return MPRK_OK;
}

int step_launches(mprk_ctx* c, double dt)
{
    const int s = c->mb.lay.s, m = c->mb.cfg.m;
    for (int k = 1; k <= m; ++k) {
        for (int j = 1; j <= s; ++j) {
            int rc = launch(c, ctx_stage_args(c, dt, k, j));
            if (rc != MPRK_OK) return rc;
        }
    }
    return MPRK_OK;
}

// A graph of the m*s stage launches of one slow step (rebuilt when dt or the
// tile shape changes).
int ctx_graph(mprk_ctx* c, double dt)
{
    if (c->graph.exec && c->graph_dt == dt && c->graph_shape == c->shape) return MPRK_OK;
    const int s = c->mb.lay.s, m = c->mb.cfg.m, ms = m * s;
    c->g_args.clear();
    for (int k = 1; k <= m; ++k)
        for (int j = 1; j <= s; ++j) c->g_args.push_back(ctx_stage_args(c, dt, k, j));
    c->g_ptrs.resize(ms);
    if (!c->graph.begin()) return MPRK_EHIP;
    const KernelRef kr = c->mb.cfg.dim == 3 ? stage3_kernel_ref(c->mb.cfg.flux_bits == 32)
                                            : stage_kernel_ref(c->mb.cfg.flux_bits == 32, c->shape);
    hipGraphNode_t prev = nullptr;
    for (int i = 0; i < ms; ++i) {
        if (c->g_args[i].nblocks <= 0) continue;
        c->g_ptrs[i] = &c->g_args[i];
        if (!c->graph.add(kr, c->g_args[i].nblocks, &c->g_ptrs[i], &prev)) {
            c->graph.reset();
            return MPRK_EHIP;
        }
    }
    if (!c->graph.finish()) {
        c->graph.reset();
        return MPRK_EHIP;
    }
    c->graph_dt = dt;
    c->graph_shape = c->shape;
    return MPRK_OK;
}

// One persistent launch running nsteps slow steps.
int run_persistent(mprk_ctx* c, double dt, int64_t nsteps)
{
    if (c->mb.cfg.dim == 3) return MPRK_EUNSUPPORTED;
    const mprk_config& g = c->mb.cfg;
    const int ms = c->mb.ms();
    char* ws = c->mb.ws;
    const int ntiles = member_tiles(g, c->shape);
    if (c->pgrid <= 0 || c->ptiles_shape != c->shape) {
        int rc = persistent_setup(g.flux_bits == 32, c->shape, ntiles, c->wait_seconds, &c->pgrid,
                                  &c->wait_ticks);
        if (rc != MPRK_OK) {
            c->pgrid = 0;
            return rc;
        }
    }
    if (c->ptiles_shape != c->shape) {
        c->h_tiles.clear();
        persistent_member(c->mb, 0, c->shape, 0, c->h_tiles, c->h_mr);
        if (hipMemcpyAsync(ws + c->lay.off_ptiles, c->h_tiles.data(), c->h_tiles.size() * sizeof(TileRef),
                           hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return MPRK_EHIP;
        c->ptiles_shape = c->shape;
    }
    if (c->ptab_dt != dt || c->ptab_shape != c->shape) {
        std::vector<StageArgs>& tab = c->h_tab;
        tab.clear();
        for (int k = 1; k <= g.m; ++k)
            for (int j = 1; j <= c->mb.lay.s; ++j) tab.push_back(ctx_stage_args(c, dt, k, j));
        if (hipMemcpyAsync(ws + c->lay.off_ptab, tab.data(), tab.size() * sizeof(StageArgs),
                           hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return MPRK_EHIP;
        c->ptab_dt = dt;
        c->ptab_shape = c->shape;
    }
    if ((int64_t)nsteps * ms > (int64_t)(1 << 30)) return MPRK_EINVAL;
    std::vector<TileRef> scratch;
    MemberRun& mr = c->h_mr;
    persistent_member(c->mb, 0, c->shape, 0, scratch, mr);
    mr.stages = (const StageArgs*)(ws + c->lay.off_ptab);
    mr.slot_stage = nullptr;
    mr.nslots = ms;
    mr.nsteps = (int32_t)nsteps;
    if (hipMemcpyAsync(ws + c->lay.off_pmember, &mr, sizeof mr, hipMemcpyHostToDevice, c->stream) !=
        hipSuccess)
        return MPRK_EHIP;
    int32_t* done = (int32_t*)(ws + c->lay.off_pdone);
    if (launch_fill_i32(done, 0, ntiles + 1, c->stream) != hipSuccess) return MPRK_EHIP;
    PersistArgs P;
    std::memset(&P, 0, sizeof P);
    P.tiles = (const TileRef*)(ws + c->lay.off_ptiles);
    P.members = (const MemberRun*)(ws + c->lay.off_pmember);
    P.done = done;
    P.abort_flag = done + ntiles;
    P.ntiles = ntiles;
    P.gmax = (int32_t)(nsteps * ms);
    P.run_ticks = c->wait_ticks;
    if (launch_persistent(P, c->pgrid, g.flux_bits == 32, c->shape, c->stream) != hipSuccess)
        return MPRK_EHIP;
    return MPRK_OK;
}

int advance(mprk_ctx* c, double dt, int64_t nsteps)
{
    if (nsteps <= 0) return MPRK_OK;
    int rc = MPRK_OK;
    if (c->exec == MPRK_EXEC_PERSISTENT) {
        rc = run_persistent(c, dt, nsteps);
    } else if (c->exec == MPRK_EXEC_GRAPH && !c->prof_on) {
        rc = ctx_graph(c, dt);
        for (int64_t n = 0; n < nsteps && rc == MPRK_OK; ++n)
            if (hipGraphLaunch(c->graph.exec, c->stream) != hipSuccess) rc = MPRK_EHIP;
    } else {
        for (int64_t n = 0; n < nsteps && rc == MPRK_OK; ++n) rc = step_launches(c, dt);
    }
    if (rc == MPRK_OK) c->steps += nsteps;
    return rc;
}

int run_reduce(mprk_ctx* c, mprk_stats* out)
{
    int rc = member_reduce_launch(c->mb, c->stream, c->host_final);
    if (rc != MPRK_OK) return rc;
    int32_t aborted = 0;
    if (c->exec == MPRK_EXEC_PERSISTENT && c->ptiles_shape >= 0 &&
        hipMemcpyAsync(&aborted, (int32_t*)(c->mb.ws + c->lay.off_pdone) + member_tiles(c->mb.cfg, c->shape),
                       sizeof aborted, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return MPRK_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MPRK_EHIP;
    if (aborted) return MPRK_ETIMEOUT;
    return member_stats(c->mb, c->host_final, c->steps, out);
}

// ---- batches -------------------------------------------------------------

struct BatchLayout {
    std::vector<size_t> core_off;
    size_t off_tab, off_proxy, off_bmap, off_slots, off_ptiles, off_pmember, off_pdone;
    size_t off_red, off_finals;
    int nslots, total_ms, max_tiles;
    size_t total;
};

int batch_check(const mprk_member* mem, int32_t n, char* msg, size_t len)
{
    if (!mem || n < 1 || n > 4096) {
        set_msg(msg, len, "need 1..4096 members");
        return MPRK_EINVAL;
    }
    for (int i = 0; i < n; ++i) {
        char m2[160];
        const int rc = mprk_validate(&mem[i].cfg, m2, sizeof m2);
        if (rc != MPRK_OK) {
            set_msg(msg, len, "member %d: %s", i, m2);
            return rc;
        }
        if (mem[i].cfg.dim != 2) {
            set_msg(msg, len, "member %d: batches hold 2D problems", i);
            return MPRK_EUNSUPPORTED;
        }
        if (mem[i].cfg.flux_bits != mem[0].cfg.flux_bits) {
            set_msg(msg, len, "member %d: every member must use the same flux_bits", i);
            return MPRK_EINVAL;
        }
        if (!(mem[i].dt > 0) || !std::isfinite(mem[i].dt)) {
            set_msg(msg, len, "member %d: dt must be positive and finite", i);
            return MPRK_EINVAL;
        }
    }
    return MPRK_OK;
}

bool batch_layout(const mprk_member* mem, int32_t n, BatchLayout* L)
{
    L->core_off.resize(n);
    size_t off = 0;
    int ms_max = 0, total_ms = 0, tiles = 0;
    for (int i = 0; i < n; ++i) {
        CoreLayout cl;
        if (!core_layout(&mem[i].cfg, &cl)) return false;
        L->core_off[i] = off;
        off += cl.total;
        const int ms = mem[i].cfg.m * cl.s;
        ms_max = std::max(ms_max, ms);
        total_ms += ms;
        tiles += max_member_tiles(mem[i].cfg);
    }
    L->nslots = ms_max;
    L->total_ms = total_ms;
    L->max_tiles = tiles;
    L->off_tab = off;
    off += round_up((size_t)total_ms * sizeof(StageArgs));
    L->off_proxy = off;
    off += round_up((size_t)total_ms * sizeof(StageArgs));
    L->off_bmap = off;   // per slot, one entry per block (at most every member's largest tile count)
    off += round_up((size_t)ms_max * tiles * sizeof(BatchEntry));
    L->off_slots = off;
    off += round_up((size_t)ms_max * n * sizeof(int32_t));
    L->off_ptiles = off;
    off += round_up((size_t)tiles * sizeof(TileRef));
    L->off_pmember = off;
    off += round_up((size_t)n * sizeof(MemberRun));
    L->off_pdone = off;
    off += round_up((size_t)(tiles + 1) * sizeof(int32_t));
    L->off_red = off;
    off += round_up((size_t)n * sizeof(ReduceArgs));
    L->off_finals = off;
    off += round_up((size_t)n * 2 * RED_FIELDS * sizeof(double));
    L->total = off;
    return true;
}

// Stage records, slot entries and persistent tiles for the batch's shape.
// Member i's stage p (0-based within a slow step) runs in slot
// floor(p * nslots / (m_i s_i)), which spreads each member's stages evenly
// over the slow step's launches.
// Stage records only (after a change of steps; the launch layout and the
// graph, which reference the record table by address, stay valid).
// Stage record of a batch member: device-scope result stores in persistent
// mode only (9% faster there on the 64-member ensemble; launch and graph
// modes are faster with ordinary stores for batches, see st_dev).
StageArgs batch_stage_args(const mprk_batch* b, const Member& mb, int i, int k, int j)
{
    StageArgs a = stage_args(mb, b->dt[i], k, j, b->shape);
    a.dev_stores = b->exec == MPRK_EXEC_PERSISTENT ? 1 : 0;
    return a;
}

int batch_records(mprk_batch* b)
{
    b->h_tab.clear();
    b->h_proxy.clear();
    for (int i = 0; i < b->n; ++i) {
        const Member& mb = b->mb[i];
        for (int k = 1; k <= mb.cfg.m; ++k)
            for (int j = 1; j <= mb.lay.s; ++j) {
                b->h_tab.push_back(batch_stage_args(b, mb, i, k, j));
                b->h_proxy.push_back(proxy_args(mb, b->dt[i], k, j, b->shape));
            }
    }
    if (hipMemcpyAsync(b->ws + b->off_tab, b->h_tab.data(), b->h_tab.size() * sizeof(StageArgs),
                       hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipMemcpyAsync(b->ws + b->off_proxy, b->h_proxy.data(), b->h_proxy.size() * sizeof(StageArgs),
                       hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return MPRK_EHIP;
    b->rec_dirty = false;
    b->rec_dev = b->exec == MPRK_EXEC_PERSISTENT ? 1 : 0;
    return MPRK_OK;
}

int batch_tables(mprk_batch* b)
{
    if (b->tab_shape == b->shape) return b->rec_dirty ? batch_records(b) : MPRK_OK;
    const int n = b->n, L = b->nslots;
    b->h_tab.clear();
    b->h_proxy.clear();
    const size_t T = (size_t)b->max_tiles;
    b->h_bmap.assign((size_t)L * T, BatchEntry{0, 0});
    b->slot_count.assign(L, 0);
    b->slot_blocks.assign(L, 0);
    b->h_slots.assign((size_t)n * L, -1);
    for (int i = 0; i < n; ++i) {
        const Member& mb = b->mb[i];
        const int s = mb.lay.s, ms = mb.ms();
        for (int k = 1; k <= mb.cfg.m; ++k)
            for (int j = 1; j <= s; ++j) {
                b->h_tab.push_back(batch_stage_args(b, mb, i, k, j));
                b->h_proxy.push_back(proxy_args(mb, b->dt[i], k, j, b->shape));
            }
        for (int p = 0; p < ms; ++p) {
            const int slot = (int)((int64_t)p * L / ms);
            b->h_slots[(size_t)i * L + slot] = b->rec0[i] + p;
        }
    }
    for (int l = 0; l < L; ++l) {
        int blocks = 0, cnt = 0;
        for (int i = 0; i < n; ++i) {
            const int r = b->h_slots[(size_t)i * L + l];
            if (r < 0 || b->h_tab[r].nblocks <= 0) continue;
            if ((size_t)blocks + (size_t)b->h_tab[r].nblocks > T) return MPRK_EINVAL;   // cannot happen
            for (int t = 0; t < b->h_tab[r].nblocks; ++t)
                b->h_bmap[(size_t)l * T + blocks + t] = BatchEntry{r, blocks};
            blocks += b->h_tab[r].nblocks;
            ++cnt;
        }
        b->slot_count[l] = cnt;
        b->slot_blocks[l] = blocks;
    }
    b->h_tiles.clear();
    b->h_mr.assign(n, MemberRun{});
    int done = 0;
    for (int i = 0; i < n; ++i) {
        persistent_member(b->mb[i], i, b->shape, done, b->h_tiles, b->h_mr[i]);
        done += member_tiles(b->mb[i].cfg, b->shape);
        MemberRun& mr = b->h_mr[i];
        mr.stages = (const StageArgs*)(b->ws + b->off_tab) + b->rec0[i];
        // Slot table of this member, as indices relative to its own records.
        mr.slot_stage = (const int32_t*)(b->ws + b->off_slots) + (size_t)i * L;
        mr.nslots = L;
    }
    for (int i = 0; i < n; ++i)
        for (int l = 0; l < L; ++l) {
            int32_t& r = b->h_slots[(size_t)i * L + l];
            if (r >= 0) r -= b->rec0[i];
        }
    hipStream_t st = b->stream;
    if (hipMemcpyAsync(b->ws + b->off_tab, b->h_tab.data(), b->h_tab.size() * sizeof(StageArgs),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->ws + b->off_proxy, b->h_proxy.data(), b->h_proxy.size() * sizeof(StageArgs),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->ws + b->off_bmap, b->h_bmap.data(), b->h_bmap.size() * sizeof(BatchEntry),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->ws + b->off_slots, b->h_slots.data(), b->h_slots.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->ws + b->off_ptiles, b->h_tiles.data(), b->h_tiles.size() * sizeof(TileRef),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return MPRK_EHIP;
    b->tab_shape = b->shape;
    b->rec_dirty = false;
    b->rec_dev = b->exec == MPRK_EXEC_PERSISTENT ? 1 : 0;
    b->graph.reset();           // block counts per launch may differ for a new shape
    return MPRK_OK;
}

// The slot launches of one slow step (proxy: the autotuner's workload).
int batch_step_launches(mprk_batch* b, bool proxy)
{
    const StageArgs* tab = (const StageArgs*)(b->ws + (proxy ? b->off_proxy : b->off_tab));
    const BatchEntry* bmap = (const BatchEntry*)(b->ws + b->off_bmap);
    for (int l = 0; l < b->nslots; ++l) {
        if (b->slot_count[l] == 0) continue;
        if (launch_batch(tab, bmap + (size_t)l * b->max_tiles, b->slot_blocks[l], b->flux32, b->shape,
                         b->stream) != hipSuccess)
            return MPRK_EHIP;
    }
    return MPRK_OK;
}

int batch_graph(mprk_batch* b)
{
    if (b->graph.exec && b->graph_shape == b->shape) return MPRK_OK;
    const int L = b->nslots;
    b->g_vals.assign(L, mprk_batch::NodeArgs{});
    b->g_args.assign(L, std::vector<void*>(3, nullptr));
    if (!b->graph.begin()) return MPRK_EHIP;
    const KernelRef kr = batch_kernel_ref(b->flux32, b->shape);
    hipGraphNode_t prev = nullptr;
    for (int l = 0; l < L; ++l) {
        if (b->slot_count[l] == 0) continue;
        mprk_batch::NodeArgs& v = b->g_vals[l];
        v.tab = (const StageArgs*)(b->ws + b->off_tab);
        v.bmap = (const BatchEntry*)(b->ws + b->off_bmap) + (size_t)l * b->max_tiles;
        v.nblocks = b->slot_blocks[l];
        std::vector<void*>& a = b->g_args[l];
        a[0] = &v.tab;
        a[1] = &v.bmap;
        a[2] = &v.nblocks;
        if (!b->graph.add(kr, v.nblocks, a.data(), &prev)) {
            b->graph.reset();
            return MPRK_EHIP;
        }
    }
    if (!b->graph.finish()) {
        b->graph.reset();
        return MPRK_EHIP;
    }
    b->graph_shape = b->shape;
    return MPRK_OK;
}

int batch_persistent(mprk_batch* b, int64_t nsteps)
{
    int ntiles = 0;
    for (int i = 0; i < b->n; ++i) ntiles += member_tiles(b->mb[i].cfg, b->shape);
    if (b->pgrid <= 0 || b->pgrid_shape != b->shape) {
        int rc = persistent_setup(b->flux32, b->shape, ntiles, b->wait_seconds, &b->pgrid, &b->wait_ticks);
        if (rc != MPRK_OK) {
            b->pgrid = 0;
            return rc;
        }
        b->pgrid_shape = b->shape;
    }
    if ((int64_t)nsteps * b->nslots > (int64_t)(1 << 30)) return MPRK_EINVAL;
    for (int i = 0; i < b->n; ++i) b->h_mr[i].nsteps = (int32_t)nsteps;
    if (hipMemcpyAsync(b->ws + b->off_pmember, b->h_mr.data(), b->h_mr.size() * sizeof(MemberRun),
                       hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return MPRK_EHIP;
    int32_t* done = (int32_t*)(b->ws + b->off_pdone);
    if (launch_fill_i32(done, 0, ntiles + 1, b->stream) != hipSuccess) return MPRK_EHIP;
    PersistArgs P;
    std::memset(&P, 0, sizeof P);
    P.tiles = (const TileRef*)(b->ws + b->off_ptiles);
    P.members = (const MemberRun*)(b->ws + b->off_pmember);
    P.done = done;
    P.abort_flag = done + ntiles;
    P.ntiles = ntiles;
    P.gmax = (int32_t)(nsteps * b->nslots);
    P.run_ticks = b->wait_ticks;
    if (launch_persistent(P, b->pgrid, b->flux32, b->shape, b->stream) != hipSuccess) return MPRK_EHIP;
    return MPRK_OK;
}

int batch_advance(mprk_batch* b, int64_t nsteps)
{
    if (nsteps <= 0) return MPRK_OK;
    int rc = batch_tables(b);
    if (rc != MPRK_OK) return rc;
    if (b->exec == MPRK_EXEC_PERSISTENT) {
        rc = batch_persistent(b, nsteps);
    } else if (b->exec == MPRK_EXEC_GRAPH) {
        rc = batch_graph(b);
        for (int64_t k = 0; k < nsteps && rc == MPRK_OK; ++k)
            if (hipGraphLaunch(b->graph.exec, b->stream) != hipSuccess) rc = MPRK_EHIP;
    } else {
        for (int64_t k = 0; k < nsteps && rc == MPRK_OK; ++k) rc = batch_step_launches(b, false);
    }
    if (rc == MPRK_OK) b->steps += nsteps;
    return rc;
}

// Reductions of every member in two launches and one copy back.
int batch_reduce(mprk_batch* b, mprk_stats* out)
{
    const int n = b->n;
    const size_t nf = (size_t)n * 2 * RED_FIELDS;
    b->host_final.resize(nf);
    double* finals = (double*)(b->ws + b->off_finals);
    if (!b->red_ready) {
        b->h_red.resize(n);
        for (int i = 0; i < n; ++i) b->h_red[i] = member_reduce_args(b->mb[i], finals + (size_t)i * 2 * RED_FIELDS);
        if (hipMemcpyAsync(b->ws + b->off_red, b->h_red.data(), n * sizeof(ReduceArgs), hipMemcpyHostToDevice,
                           b->stream) != hipSuccess)
            return MPRK_EHIP;
        b->red_ready = true;
    }
    if (launch_reduce_batch((const ReduceArgs*)(b->ws + b->off_red), n, b->stream) != hipSuccess)
        return MPRK_EHIP;
    if (hipMemcpyAsync(b->host_final.data(), finals, nf * sizeof(double), hipMemcpyDeviceToHost, b->stream) !=
        hipSuccess)
        return MPRK_EHIP;
    int32_t aborted = 0;
    if (b->exec == MPRK_EXEC_PERSISTENT && b->tab_shape >= 0) {
        int ntiles = 0;
        for (int i = 0; i < n; ++i) ntiles += member_tiles(b->mb[i].cfg, b->shape);
        if (hipMemcpyAsync(&aborted, (int32_t*)(b->ws + b->off_pdone) + ntiles, sizeof aborted,
                           hipMemcpyDeviceToHost, b->stream) != hipSuccess)
            return MPRK_EHIP;
    }
    if (hipStreamSynchronize(b->stream) != hipSuccess) return MPRK_EHIP;
    if (aborted) return MPRK_ETIMEOUT;
    int worst = MPRK_OK;
    for (int i = 0; i < n; ++i) {
        const int rc = member_stats(b->mb[i], b->host_final.data() + (size_t)i * 2 * RED_FIELDS, b->steps,
                                    out ? out + i : nullptr);
        if (rc != MPRK_OK) worst = rc;
    }
    return worst;
}

}  // namespace

extern "C" {

const char* mprk_strerror(int code)
{
    switch (code) {
    case MPRK_OK: return "ok";
    case MPRK_EINVAL: return "invalid configuration or argument";
    case MPRK_EBUFFER: return "buffer shorter than 2s-1 rows (strict_buffer)";
    case MPRK_EWORKSPACE: return "workspace missing, too small or misaligned";
    case MPRK_EHIP: return "HIP runtime error";
    case MPRK_ENONFINITE: return "non-finite or non-physical state";
    case MPRK_EUNSUPPORTED: return "not supported by the library or device";
    case MPRK_ETIMEOUT: return "a persistent-kernel wait timed out (run aborted)";
    default: return "unknown status";
    }
}

int mprk_validate(const mprk_config* c, char* msg, size_t len)
{
    set_msg(msg, len, "ok");
    if (!c) { set_msg(msg, len, "null config"); return MPRK_EINVAL; }
    if (c->abi_version != MPRK_ABI_VERSION) {
        set_msg(msg, len, "abi_version %d, library %d", c->abi_version, MPRK_ABI_VERSION);
        return MPRK_EINVAL;
    }
    if (c->dim != 2 && c->dim != 3) { set_msg(msg, len, "dim must be 2 or 3"); return MPRK_EINVAL; }
    if (c->dim == 2 && c->ny != 1) { set_msg(msg, len, "ny must be 1 in 2D"); return MPRK_EINVAL; }
    if (c->dim == 3 && (c->ny < 4 || !(c->dy > 0) || !std::isfinite(c->dy))) {
        set_msg(msg, len, "3D needs ny >= 4 and a positive finite dy");
        return MPRK_EINVAL;
    }
    if (c->nx < 4 || c->nz_lower < 3 || c->nz_upper < 3) {
        set_msg(msg, len, "need nx >= 4 and nz >= 3 per domain");
        return MPRK_EINVAL;
    }
    const long long ny_ = c->dim == 3 ? c->ny : 1;
    if ((long long)c->nx * ny_ * std::max(c->nz_lower, c->nz_upper) > (1LL << 28)) {
        set_msg(msg, len, "domain larger than 2^28 cells");
        return MPRK_EINVAL;
    }
    if (!(c->dx > 0) || !(c->dz_lower > 0) || !(c->dz_upper > 0) || !std::isfinite(c->dx) ||
        !std::isfinite(c->dz_lower) || !std::isfinite(c->dz_upper)) {
        set_msg(msg, len, "cell sizes must be positive and finite");
        return MPRK_EINVAL;
    }
    if (c->fast_is_lower != 0 && c->fast_is_lower != 1) {
        set_msg(msg, len, "fast_is_lower must be 0 or 1");
        return MPRK_EINVAL;
    }
    if (c->base_rk != 2 && c->base_rk != 3) {
        set_msg(msg, len, "base_rk must be 2 or 3");
        return MPRK_EINVAL;
    }
    if (c->m < 1 || c->m > 64) { set_msg(msg, len, "m must be in 1..64"); return MPRK_EINVAL; }
    const int nz_slow = c->fast_is_lower ? c->nz_upper : c->nz_lower;
    if (c->n_buffer < 1 || c->n_buffer > nz_slow - 2) {
        set_msg(msg, len, "n_buffer must be in 1..%d", nz_slow - 2);
        return MPRK_EINVAL;
    }
    if (!(c->gamma > 1.0) || !std::isfinite(c->gamma)) {
        set_msg(msg, len, "gamma must exceed 1");
        return MPRK_EINVAL;
    }
    if (!(c->prandtl > 0.0) || !std::isfinite(c->prandtl)) {
        set_msg(msg, len, "prandtl must be positive");
        return MPRK_EINVAL;
    }
    if (!(c->mu_lower > 0.0) || !(c->mu_upper > 0.0) || !std::isfinite(c->mu_lower) ||
        !std::isfinite(c->mu_upper)) {
        set_msg(msg, len, "viscosities must be positive (the bulk coupling divides by them)");
        return MPRK_EINVAL;
    }
    if (!std::isfinite(c->gravity)) { set_msg(msg, len, "gravity must be finite"); return MPRK_EINVAL; }
    if (c->flux_bits != 64 && c->flux_bits != 32) {
        set_msg(msg, len, "flux_bits must be 64 or 32");
        return MPRK_EINVAL;
    }
    const int s = c->base_rk;
    if (c->m > 1 && c->n_buffer < 2 * s - 1) {
        if (c->strict_buffer) {
            set_msg(msg, len, "n_buffer %d < 2s-1 = %d", c->n_buffer, 2 * s - 1);
            return MPRK_EBUFFER;
        }
        set_msg(msg, len, "warning: n_buffer %d < 2s-1 = %d; not exactly conservative",
                c->n_buffer, 2 * s - 1);
    }
    return MPRK_OK;
}

size_t mprk_workspace_bytes(const mprk_config* c)
{
    if (mprk_validate(c, nullptr, 0) != MPRK_OK) return 0;
    CtxLayout L;
    if (!ctx_layout(c, &L)) return 0;
    return L.total;
}

int mprk_stable_dt(const mprk_config* c, const mprk_stats* st, double cr, double dn, double* dt_out)
{
    if (!c || !st || !dt_out || !(cr > 0) || !(dn > 0)) return MPRK_EINVAL;
    if (st->status) return MPRK_ENONFINITE;
    const bool fl = c->fast_is_lower != 0;
    const double lamF = fl ? st->lambda_lower : st->lambda_upper;
    const double lamS = fl ? st->lambda_upper : st->lambda_lower;
    const double visF = fl ? st->visc_lower : st->visc_upper;
    const double visS = fl ? st->visc_upper : st->visc_lower;
    if (!(lamF > 0) || !(lamS > 0)) return MPRK_EINVAL;
    // Combined advective + diffusive limit per domain (the odd-even mode gets
    // both as real negative eigenvalue parts): 1 / (lambda/cr + visc/dn).
    const double dtf = 1.0 / (lamF / cr + visF / dn);
    const double dts = 1.0 / (lamS / cr + visS / dn);
    const double dt = std::min(c->m * dtf, dts);
    *dt_out = dt;
    return MPRK_OK;
}

int mprk_create(const mprk_config* cfg, double* q_lower, double* q_upper, void* workspace,
                size_t workspace_bytes, void* hip_stream, mprk_ctx** out)
{
    if (!out) return MPRK_EINVAL;
    *out = nullptr;
    int rc = mprk_validate(cfg, nullptr, 0);
    if (rc != MPRK_OK) return rc;
    if (!q_lower || !q_upper) return MPRK_EINVAL;
    if (((uintptr_t)q_lower | (uintptr_t)q_upper) % sizeof(double)) return MPRK_EINVAL;
    CtxLayout L;
    if (!ctx_layout(cfg, &L)) return MPRK_EINVAL;
    if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace % ALIGN))
        return MPRK_EWORKSPACE;
    mprk_ctx* c = new (std::nothrow) mprk_ctx();
    if (!c) return MPRK_EINVAL;
    c->lay = L;
    c->mb.init(*cfg, L.core, q_lower, q_upper, (char*)workspace);
    c->stream = (hipStream_t)hip_stream;
    c->shape = default_shape(*cfg);
    *out = c;
    return MPRK_OK;
}

int mprk_set_stream(mprk_ctx* c, void* s)
{
    if (!c) return MPRK_EINVAL;
    c->stream = (hipStream_t)s;
    return MPRK_OK;
}

int mprk_destroy(mprk_ctx* c)
{
    if (!c) return MPRK_EINVAL;
    hipError_t e = hipStreamSynchronize(c->stream);
    c->graph.reset();
    for (hipEvent_t ev : c->prof_ev) (void)hipEventDestroy(ev);
    delete c;
    return e == hipSuccess ? MPRK_OK : MPRK_EHIP;
}

int mprk_rhs(mprk_ctx* c, const double* q_lower, const double* q_upper, double* r_lower,
             double* r_upper, int mask)
{
    if (!c || !q_lower || !q_upper || !r_lower || !r_upper) return MPRK_EINVAL;
    if (mask & ~MPRK_REGION_ALL) return MPRK_EINVAL;
    const Member& mb = c->mb;
    const mprk_config& g = mb.cfg;
    StageArgs a = base_args(mb);
    const double* qs[2] = {q_lower, q_upper};
    double* rs[2] = {r_lower, r_upper};
    for (int d = 0; d < 2; ++d) {
        DomainArgs& D = a.d[d];
        D.qin = qs[d];
        D.base = qs[d];
        D.out = rs[d];
        D.main = combine(0.0, 0.0, MODE_RHS);
        D.buf = D.main;
        int lo = 0, hi = 0;
        if (d == mb.fast) {
            if (mask & MPRK_REGION_F) hi = D.nz;
        } else {
            const bool wb = mask & MPRK_REGION_B, ws = mask & MPRK_REGION_S;
            if (wb && ws) { lo = 0; hi = D.nz; }
            else if (wb) { lo = mb.b_lo; hi = mb.b_hi; }
            else if (ws) {
                if (g.fast_is_lower) { lo = mb.b_hi; hi = D.nz; }
                else { lo = 0; hi = mb.b_lo; }
            }
        }
        set_rows(D, g, lo, hi, c->shape);
    }
    finish_record(mb, a);
    return launch(c, a);
}

int mprk_set_exec(mprk_ctx* c, int mode)
{
    if (!c || !valid_mode(mode)) return MPRK_EINVAL;
    if (c->mb.cfg.dim == 3 && mode == MPRK_EXEC_PERSISTENT) return MPRK_EUNSUPPORTED;
    c->exec = mode;
    return MPRK_OK;
}

int mprk_set_tile(mprk_ctx* c, int shape)
{
    if (!c || shape < 0 || shape >= MPRK_TILE_SHAPES) return MPRK_EINVAL;
    if (c->mb.cfg.dim == 3 && shape != MPRK_TILE_32X16) return MPRK_EUNSUPPORTED;
    c->shape = shape;
    return MPRK_OK;
}

int mprk_set_wait_limit(mprk_ctx* c, double seconds)
{
    if (!c || !(seconds >= 0.0) || !(seconds <= 3600.0)) return MPRK_EINVAL;
    c->wait_seconds = seconds;
    c->pgrid = 0;   // recompute the tick limit at the next persistent launch
    return MPRK_OK;
}

int mprk_step(mprk_ctx* c, double dt)
{
    if (!c || !(dt > 0) || !std::isfinite(dt)) return MPRK_EINVAL;
    return advance(c, dt, 1);
}

int mprk_profile_enable(mprk_ctx* c, int on)
{
    if (!c) return MPRK_EINVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MPRK_EHIP;
    c->prof_on = on != 0;
    c->prof_used = 0;
    return MPRK_OK;
}

int mprk_profile_take(mprk_ctx* c, double* kernel_ms, int64_t* launches)
{
    if (!c || !kernel_ms || !launches) return MPRK_EINVAL;
    double tot = 0.0;
    if (c->prof_used > 0) {
        if (hipEventSynchronize(c->prof_ev[2 * c->prof_used - 1]) != hipSuccess) return MPRK_EHIP;
        for (size_t i = 0; i < c->prof_used; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]) != hipSuccess)
                return MPRK_EHIP;
            tot += ms;
        }
    }
    *kernel_ms = tot;
    *launches = (int64_t)c->prof_used;
    c->prof_used = 0;
    return MPRK_OK;
}

int mprk_diagnostics(mprk_ctx* c, mprk_stats* out)
{
    if (!c) return MPRK_EINVAL;
    return run_reduce(c, out);
}

int mprk_diagnostics_static(const mprk_config* cfg, const double* q_lower, const double* q_upper,
                            void* hip_stream, mprk_stats* out)
{
    const int rc = mprk_validate(cfg, nullptr, 0);
    if (rc != MPRK_OK) return rc;
    if (!q_lower || !q_upper) return MPRK_EINVAL;
    if (((uintptr_t)q_lower | (uintptr_t)q_upper) % sizeof(double)) return MPRK_EINVAL;
    // The scratch need is fixed (partials of a fixed block count, then the
    // finals) whatever the size mprk_validate accepted.
    static_assert(STATIC_SCRATCH_DOUBLES >= (size_t)2 * RED_BLOCKS * RED_FIELDS + 2 * RED_FIELDS,
                  "scratch holds the partials and the finals");
    double* scr = nullptr;
    if (static_scratch_address(&scr) != hipSuccess) return MPRK_EHIP;
    const hipStream_t stream = (hipStream_t)hip_stream;
    const ReduceArgs r = reduce_args(*cfg, q_lower, q_upper, scr, scr + (size_t)2 * RED_BLOCKS * RED_FIELDS);
    if (launch_reduce(r, stream) != hipSuccess) return MPRK_EHIP;
    double host_final[2 * RED_FIELDS];
    if (hipMemcpyAsync(host_final, r.final_, sizeof host_final, hipMemcpyDeviceToHost, stream) != hipSuccess)
        return MPRK_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return MPRK_EHIP;
    return stats_from_final(*cfg, host_final, 0, out);
}

int mprk_run(mprk_ctx* c, double dt, int64_t nsteps, int64_t check_every, mprk_stats* out)
{
    if (!c || nsteps < 0) return MPRK_EINVAL;
    if (nsteps > 0 && (!(dt > 0) || !std::isfinite(dt))) return MPRK_EINVAL;
    if (nsteps == 0) return run_reduce(c, out);
    const int64_t chunk = check_every > 0 ? check_every : nsteps;
    for (int64_t done = 0; done < nsteps;) {
        const int64_t n = std::min(chunk, nsteps - done);
        int rc = advance(c, dt, n);
        if (rc != MPRK_OK) return rc;
        done += n;
        rc = run_reduce(c, out);
        if (rc != MPRK_OK) return rc;
    }
    return MPRK_OK;
}

// ---- batches ---------------------------------------------------------------

int mprk_batch_validate(const mprk_member* members, int32_t n, char* msg, size_t len)
{
    return batch_check(members, n, msg, len);
}

size_t mprk_batch_workspace_bytes(const mprk_member* members, int32_t n)
{
    if (batch_check(members, n, nullptr, 0) != MPRK_OK) return 0;
    BatchLayout L;
    if (!batch_layout(members, n, &L)) return 0;
    return L.total;
}

int mprk_batch_create(const mprk_member* members, int32_t n, void* workspace, size_t workspace_bytes,
                      void* hip_stream, mprk_batch** out)
{
    if (!out) return MPRK_EINVAL;
    *out = nullptr;
    int rc = batch_check(members, n, nullptr, 0);
    if (rc != MPRK_OK) return rc;
    // States must be distinct, non-overlapping device arrays.
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    for (int i = 0; i < n; ++i) {
        const mprk_config& g = members[i].cfg;
        const double* q[2] = {members[i].q_lower, members[i].q_upper};
        const size_t len[2] = {(size_t)NV * g.nz_lower * g.nx * 8, (size_t)NV * g.nz_upper * g.nx * 8};
        for (int d = 0; d < 2; ++d) {
            if (!q[d] || (uintptr_t)q[d] % sizeof(double)) return MPRK_EINVAL;
            spans.push_back({(uintptr_t)q[d], (uintptr_t)q[d] + len[d]});
        }
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return MPRK_EINVAL;
    BatchLayout L;
    if (!batch_layout(members, n, &L)) return MPRK_EINVAL;
    if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace % ALIGN)) return MPRK_EWORKSPACE;
    mprk_batch* b = new (std::nothrow) mprk_batch();
    if (!b) return MPRK_EINVAL;
    b->n = n;
    b->ws = (char*)workspace;
    b->stream = (hipStream_t)hip_stream;
    b->flux32 = members[0].cfg.flux_bits == 32;
    b->shape = default_shape(members[0].cfg);
    b->mb.resize(n);
    b->dt.resize(n);
    b->rec0.resize(n);
    int rec = 0;
    for (int i = 0; i < n; ++i) {
        CoreLayout cl;
        core_layout(&members[i].cfg, &cl);
        b->mb[i].init(members[i].cfg, cl, members[i].q_lower, members[i].q_upper,
                      b->ws + L.core_off[i]);
        b->dt[i] = members[i].dt;
        b->rec0[i] = rec;
        rec += b->mb[i].ms();
    }
    b->nslots = L.nslots;
    b->total_ms = L.total_ms;
    b->max_tiles = L.max_tiles;
    b->off_tab = L.off_tab;
    b->off_proxy = L.off_proxy;
    b->off_bmap = L.off_bmap;
    b->off_slots = L.off_slots;
    b->off_ptiles = L.off_ptiles;
    b->off_pmember = L.off_pmember;
    b->off_pdone = L.off_pdone;
    b->off_red = L.off_red;
    b->off_finals = L.off_finals;
    *out = b;
    return MPRK_OK;
}

int mprk_batch_set_exec(mprk_batch* b, int mode)
{
    if (!b || !valid_mode(mode)) return MPRK_EINVAL;
    b->exec = mode;
    if ((mode == MPRK_EXEC_PERSISTENT ? 1 : 0) != b->rec_dev) b->rec_dirty = true;   // store policy
    return MPRK_OK;
}

int mprk_batch_set_tile(mprk_batch* b, int shape)
{
    if (!b || shape < 0 || shape >= MPRK_TILE_SHAPES) return MPRK_EINVAL;
    b->shape = shape;
    return MPRK_OK;
}

int mprk_batch_set_dt(mprk_batch* b, int32_t member, double dt)
{
    if (!b || member < 0 || member >= b->n || !(dt > 0) || !std::isfinite(dt)) return MPRK_EINVAL;
    if (b->dt[member] != dt) {
        b->dt[member] = dt;
        b->rec_dirty = true;    // stage records carry dt
    }
    return MPRK_OK;
}

int mprk_batch_set_wait_limit(mprk_batch* b, double seconds)
{
    if (!b || !(seconds >= 0.0) || !(seconds <= 3600.0)) return MPRK_EINVAL;
    b->wait_seconds = seconds;
    b->pgrid = 0;
    return MPRK_OK;
}

int mprk_batch_tune(mprk_batch* b, int32_t reps, double* ms_out, int32_t* best)
{
    if (!b || reps < 1 || reps > 1000) return MPRK_EINVAL;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MPRK_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MPRK_EHIP;
    }
    const int keep = b->shape;
    int rc = MPRK_OK, pick = keep;
    double best_ms = 0.0;
    for (int sh = 0; sh < MPRK_TILE_SHAPES && rc == MPRK_OK; ++sh) {
        b->shape = sh;
        rc = batch_tables(b);
        if (rc == MPRK_OK) rc = batch_step_launches(b, true);   // warm-up
        if (rc == MPRK_OK && hipEventRecord(e0, b->stream) != hipSuccess) rc = MPRK_EHIP;
        for (int r = 0; r < reps && rc == MPRK_OK; ++r) rc = batch_step_launches(b, true);
        if (rc == MPRK_OK && hipEventRecord(e1, b->stream) != hipSuccess) rc = MPRK_EHIP;
        float ms = 0.0f;
        if (rc == MPRK_OK && (hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = MPRK_EHIP;
        if (rc != MPRK_OK) break;
        const double per = (double)ms / reps;
        if (ms_out) ms_out[sh] = per;
        if (sh == 0 || per < best_ms) {
            best_ms = per;
            pick = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->shape = rc == MPRK_OK ? pick : keep;
    if (best) *best = b->shape;
    return rc;
}

int mprk_batch_set_adaptive(mprk_batch* b, double cr, double dn)
{
    if (!b || !(cr >= 0.0) || !std::isfinite(cr) || (cr > 0.0 && !(dn > 0.0 && std::isfinite(dn))))
        return MPRK_EINVAL;
    b->adapt_cr = cr;
    b->adapt_dn = dn;
    return MPRK_OK;
}

int mprk_batch_get_dt(mprk_batch* b, int32_t member, double* dt)
{
    if (!b || !dt || member < 0 || member >= b->n) return MPRK_EINVAL;
    *dt = b->dt[member];
    return MPRK_OK;
}

int mprk_batch_run(mprk_batch* b, int64_t nsteps, int64_t check_every, mprk_stats* out)
{
    if (!b || nsteps < 0) return MPRK_EINVAL;
    b->chk.resize(b->n);
    if (nsteps == 0) return batch_reduce(b, out);
    const int64_t chunk = check_every > 0 ? check_every : nsteps;
    for (int64_t done = 0; done < nsteps;) {
        const int64_t k = std::min(chunk, nsteps - done);
        int rc = batch_advance(b, k);
        if (rc != MPRK_OK) return rc;
        done += k;
        rc = batch_reduce(b, b->chk.data());
        if (out) std::copy(b->chk.begin(), b->chk.end(), out);
        if (rc != MPRK_OK) return rc;
        if (b->adapt_cr > 0.0) {
            // Each member's next step from its own state: a member's step
            // sequence does not depend on the rest of the batch.
            for (int i = 0; i < b->n; ++i) {
                double dt = 0.0;
                rc = mprk_stable_dt(&b->mb[i].cfg, &b->chk[i], b->adapt_cr, b->adapt_dn, &dt);
                if (rc != MPRK_OK) return rc;
                rc = mprk_batch_set_dt(b, i, dt);
                if (rc != MPRK_OK) return rc;
            }
        }
    }
    return MPRK_OK;
}

int mprk_batch_diagnostics(mprk_batch* b, mprk_stats* out)
{
    if (!b) return MPRK_EINVAL;
    return batch_reduce(b, out);
}

int mprk_batch_destroy(mprk_batch* b)
{
    if (!b) return MPRK_EINVAL;
    hipError_t e = hipStreamSynchronize(b->stream);
    b->graph.reset();
    delete b;
    return e == hipSuccess ? MPRK_OK : MPRK_EHIP;
}

}  // extern "C"
