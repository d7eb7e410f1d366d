// mprk_host.cpp -- host side of the MPRK library: configuration checks,
// workspace layout, the stage schedule of one slow step (Algorithm 1 in a
// low-storage substep form) and the device reductions.
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

struct Layout {
    int s;
    size_t n_lo, n_up;        // doubles per state array
    size_t off_stage_lo[3];   // stage arrays Q_2..Q_s of each domain
    size_t off_stage_up[3];
    size_t off_ret[3];        // retained slow rows per base stage
    size_t off_acc;
    size_t off_partial, off_final;
    size_t off_ptab;          // persistent execution: stage table
    size_t off_ptiles;        //   tile table
    size_t off_pmember;       //   member record
    size_t off_pdone;         //   progress counters, then the abort flag
    int ntiles;               // fixed tiles of both domains
    size_t total;
};

bool layout_of(const mprk_config* c, Layout* L)
{
    double al[3];
    int s = shu_osher(c->base_rk, al);
    if (s < 0) return false;
    L->s = s;
    L->n_lo = (size_t)NV * c->nz_lower * c->nx;
    L->n_up = (size_t)NV * c->nz_upper * c->nx;
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
        if (multi) off += round_up((size_t)NV * 2 * c->nx * sizeof(double));
    }
    L->off_acc = off;
    if (multi) off += round_up((size_t)NV * c->n_buffer * c->nx * sizeof(double));
    L->off_partial = off;
    off += round_up((size_t)2 * RED_BLOCKS * RED_FIELDS * sizeof(double));
    L->off_final = off;
    off += round_up((size_t)2 * RED_FIELDS * sizeof(double));
    const int tiles_x = (c->nx + TX - 1) / TX;
    L->ntiles = tiles_x * ((c->nz_lower + TZ - 1) / TZ + (c->nz_upper + TZ - 1) / TZ);
    L->off_ptab = off;
    off += round_up((size_t)c->m * s * sizeof(StageArgs));
    L->off_ptiles = off;
    off += round_up((size_t)L->ntiles * sizeof(TileRef));
    L->off_pmember = off;
    off += round_up(sizeof(MemberRun));
    L->off_pdone = off;
    off += round_up((size_t)(L->ntiles + 1) * sizeof(int32_t));
    L->total = off;
    return true;
}

}  // namespace

struct mprk_ctx {
    mprk_config cfg;
    Layout lay;
    double* q[2];           // lower, upper (caller-owned device memory)
    char* ws;               // workspace base (device)
    hipStream_t stream;
    double alpha[3];
    int fast, slow;         // domain indices
    int b_lo, b_hi, ret_lo; // buffer rows and retained rows of the slow domain
    int64_t steps;
    double host_final[2 * RED_FIELDS];
    int exec = MPRK_EXEC_LAUNCH;
    double ptab_dt = 0.0;                     // dt of the uploaded stage table (0: none)
    bool ptiles_ready = false;
    int pgrid = 0;                            // persistent grid size
    int64_t wait_ticks = 0;
    double wait_seconds = 2.0;
    // Host copies of the persistent tables (the asynchronous uploads read them).
    std::vector<StageArgs> h_tab;
    std::vector<TileRef> h_tiles;
    MemberRun h_mr;
    bool prof_on = false;
    size_t prof_used = 0;                     // event pairs recorded since the last take
    std::vector<hipEvent_t> prof_ev;          // start/stop pairs, reused

    double* stage(int dom, int j)   // Q_{j+1}, j = 1..s-1 (0-based j-1)
    {
        return (double*)(ws + (dom == 0 ? lay.off_stage_lo[j - 1] : lay.off_stage_up[j - 1]));
    }
    double* ret(int j) { return (double*)(ws + lay.off_ret[j]); }
    double* acc() { return (double*)(ws + lay.off_acc); }
};

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
    case MPRK_EUNSUPPORTED: return "not supported by this build or device";
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
    if (c->dim == 3) { set_msg(msg, len, "dim 3 is not implemented"); return MPRK_EUNSUPPORTED; }
    if (c->dim != 2) { set_msg(msg, len, "dim must be 2"); return MPRK_EINVAL; }
    if (c->ny != 1) { set_msg(msg, len, "ny must be 1 in 2D"); return MPRK_EINVAL; }
    if (c->nx < 4 || c->nz_lower < 3 || c->nz_upper < 3) {
        set_msg(msg, len, "need nx >= 4 and nz >= 3 per domain");
        return MPRK_EINVAL;
    }
    if ((long long)c->nx * std::max(c->nz_lower, c->nz_upper) > (1LL << 28)) {
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
    Layout L;
    if (!layout_of(c, &L)) return 0;
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
    Layout L;
    if (!layout_of(cfg, &L)) return MPRK_EINVAL;
    if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace % ALIGN))
        return MPRK_EWORKSPACE;
    mprk_ctx* c = new (std::nothrow) mprk_ctx();
    if (!c) return MPRK_EINVAL;
    c->cfg = *cfg;
    c->lay = L;
    c->q[0] = q_lower;
    c->q[1] = q_upper;
    c->ws = (char*)workspace;
    c->stream = (hipStream_t)hip_stream;
    shu_osher(cfg->base_rk, c->alpha);
    c->fast = cfg->fast_is_lower ? 0 : 1;
    c->slow = 1 - c->fast;
    const int nzs = cfg->fast_is_lower ? cfg->nz_upper : cfg->nz_lower;
    if (cfg->fast_is_lower) {
        c->b_lo = 0;
        c->b_hi = cfg->n_buffer;
        c->ret_lo = cfg->n_buffer;
    } else {
        c->b_lo = nzs - cfg->n_buffer;
        c->b_hi = nzs;
        c->ret_lo = c->b_lo - 2;
    }
    c->steps = 0;
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
    for (hipEvent_t ev : c->prof_ev) (void)hipEventDestroy(ev);
    delete c;
    return e == hipSuccess ? MPRK_OK : MPRK_EHIP;
}

}  // extern "C"

namespace {

// Shared per-launch constants; domain-specific fields are filled by callers.
StageArgs base_args(const mprk_ctx* c)
{
    const mprk_config& g = c->cfg;
    StageArgs a;
    std::memset(&a, 0, sizeof a);
    a.nx = g.nx;
    a.dx = g.dx;
    a.inv_dx = 1.0 / g.dx;
    a.gamma = g.gamma;
    a.gm1 = g.gamma - 1.0;
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
        D.mu = d == 0 ? mu1 : mu2;
        D.kappa = d == 0 ? k1 : k2;
        D.gamma_top = d == 0;
        D.gamma_bot = d == 1;
        D.b_lo = D.b_hi = 0;
        D.ret_lo = 0;
    }
    return a;
}

void set_rows(DomainArgs& D, int nx, int lo, int hi)
{
    D.row_lo = lo;
    D.row_hi = hi;
    D.tiles_x = (nx + TX - 1) / TX;
    D.tiles_z = hi > lo ? (hi - 1) / TZ - lo / TZ + 1 : 0;   // fixed tiles meeting [lo, hi)
    D.ntiles = D.tiles_x * D.tiles_z;
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

int launch(mprk_ctx* c, StageArgs& a)
{
    a.nblocks = a.d[0].ntiles + a.d[1].ntiles;
    // Launches that cover only the buffer band of the slow domain put its
    // (short) tiles first, so they run in the first wave of workgroups.
    a.first = (a.d[c->slow].use_ret) ? c->slow : 0;
    if (!c->prof_on) return launch_stage(a, c->stream) == hipSuccess ? MPRK_OK : MPRK_EHIP;
    if (2 * c->prof_used + 2 > c->prof_ev.size()) {
        for (int i = 0; i < 2; ++i) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) return MPRK_EHIP;
            c->prof_ev.push_back(ev);
        }
    }
    hipEvent_t e0 = c->prof_ev[2 * c->prof_used], e1 = c->prof_ev[2 * c->prof_used + 1];
    if (hipEventRecord(e0, c->stream) != hipSuccess) return MPRK_EHIP;
    if (launch_stage(a, c->stream) != hipSuccess) return MPRK_EHIP;
    if (hipEventRecord(e1, c->stream) != hipSuccess) return MPRK_EHIP;
    c->prof_used += 1;
    return MPRK_OK;
}

}  // namespace

extern "C" {

int mprk_rhs(mprk_ctx* c, const double* q_lower, const double* q_upper, double* r_lower,
             double* r_upper, int mask)
{
    if (!c || !q_lower || !q_upper || !r_lower || !r_upper) return MPRK_EINVAL;
    if (mask & ~MPRK_REGION_ALL) return MPRK_EINVAL;
    const mprk_config& g = c->cfg;
    StageArgs a = base_args(c);
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
        if (d == c->fast) {
            if (mask & MPRK_REGION_F) hi = D.nz;
        } else {
            const bool wb = mask & MPRK_REGION_B, ws = mask & MPRK_REGION_S;
            if (wb && ws) { lo = 0; hi = D.nz; }
            else if (wb) { lo = c->b_lo; hi = c->b_hi; }
            else if (ws) {
                if (g.fast_is_lower) { lo = c->b_hi; hi = D.nz; }
                else { lo = 0; hi = c->b_lo; }
            }
        }
        set_rows(D, g.nx, lo, hi);
    }
    return launch(c, a);
}

}  // extern "C"

namespace {

// Launch parameters of global stage (k, j) of a slow step of size dt
// (Algorithm 1 in the low-storage substep form).
StageArgs stage_args(mprk_ctx* c, double dt, int k, int j)
{
    const mprk_config& g = c->cfg;
    const int s = c->lay.s, m = g.m;
    const int F = c->fast, S = c->slow;
    double* qF = c->q[F];
    double* qS = c->q[S];
    const int nzF = F == 0 ? g.nz_lower : g.nz_upper;
    const int nzS = S == 0 ? g.nz_lower : g.nz_upper;
    const double hF = dt / m;
    StageArgs a = base_args(c);
    const double al = c->alpha[j - 1];
    const bool last = (j == s);

    // Fast domain: m substeps of dt/m of the base method.
    DomainArgs& DF = a.d[F];
    DF.qin = (j == 1) ? qF : c->stage(F, j - 1);
    DF.base = qF;
    DF.out = last ? qF : c->stage(F, j);
    DF.main = combine(al, hF, MODE_STAGE);
    DF.buf = DF.main;
    set_rows(DF, g.nx, 0, nzF);

    // Slow domain.
    DomainArgs& DS = a.d[S];
    DS.qin = (j == 1) ? qS : c->stage(S, j - 1);
    DS.base = qS;
    DS.out = last ? qS : c->stage(S, j);
    if (m == 1) {
        // Single rate: buffer and slow rows are the same base step.
        DS.main = combine(al, dt, MODE_STAGE);
        DS.buf = DS.main;
        set_rows(DS, g.nx, 0, nzS);
    } else {
        DS.b_lo = c->b_lo;
        DS.b_hi = c->b_hi;
        DS.ret_lo = c->ret_lo;
        DS.acc = c->acc();
        // Buffer: each substep restarts from q^B_n with the full step; the
        // results of the m trial steps are averaged.
        int bmode = MODE_STAGE;
        if (last) bmode = (k == 1) ? MODE_ACC_FIRST : (k < m ? MODE_ACC_ADD : MODE_ACC_FINAL);
        DS.buf = combine(al, dt, bmode);
        DS.main = combine(al, dt, MODE_STAGE);
        if (k == 1) {
            // Slow rows: one base step; keep the two rows next to the buffer of
            // each stage value for the later substeps.
            DS.ret_out = c->ret(j - 1);
            set_rows(DS, g.nx, 0, nzS);
        } else {
            DS.use_ret = 1;
            DS.ret_in = c->ret(j - 1);
            set_rows(DS, g.nx, c->b_lo, c->b_hi);
        }
    }
    return a;
}

int step_launches(mprk_ctx* c, double dt)
{
    const int s = c->lay.s, m = c->cfg.m;
    for (int k = 1; k <= m; ++k) {
        for (int j = 1; j <= s; ++j) {
            StageArgs a = stage_args(c, dt, k, j);
            int rc = launch(c, a);
            if (rc != MPRK_OK) return rc;
        }
    }
    return MPRK_OK;
}

// One persistent launch running nsteps slow steps.
int run_persistent(mprk_ctx* c, double dt, int64_t nsteps)
{
    const mprk_config& g = c->cfg;
    const int s = c->lay.s, m = g.m, ms = m * s;
    char* ws = c->ws;
    if (c->pgrid <= 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return MPRK_EHIP;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MPRK_EHIP;
        int coop = 0;
        if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop)
            return MPRK_EUNSUPPORTED;
        const int per_cu = persistent_blocks_per_cu(g.flux_bits == 32);
        if (per_cu <= 0) return MPRK_EHIP;
        int grid = per_cu * prop.multiProcessorCount;
        if (grid > c->lay.ntiles) grid = c->lay.ntiles;
        c->pgrid = grid;
        int rate_khz = 0;
        if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
            rate_khz <= 0)
            rate_khz = 100000;
        c->wait_ticks = (int64_t)((double)rate_khz * 1000.0 * c->wait_seconds);
    }
    if (!c->ptiles_ready) {
        const int tiles_x = (g.nx + TX - 1) / TX;
        const int tz[2] = {(g.nz_lower + TZ - 1) / TZ, (g.nz_upper + TZ - 1) / TZ};
        std::vector<TileRef>& tiles = c->h_tiles;
        tiles.clear();
        tiles.reserve(c->lay.ntiles);
        for (int d = 0; d < 2; ++d)
            for (int z = 0; z < tz[d]; ++z)
                for (int x = 0; x < tiles_x; ++x) tiles.push_back(TileRef{0, d, x, z});
        if (hipMemcpyAsync(ws + c->lay.off_ptiles, tiles.data(), tiles.size() * sizeof(TileRef),
                           hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return MPRK_EHIP;
        c->ptiles_ready = true;
    }
    if (c->ptab_dt != dt) {
        std::vector<StageArgs>& tab = c->h_tab;
        tab.clear();
        tab.reserve(ms);
        for (int k = 1; k <= m; ++k)
            for (int j = 1; j <= s; ++j) tab.push_back(stage_args(c, dt, k, j));
        if (hipMemcpyAsync(ws + c->lay.off_ptab, tab.data(), tab.size() * sizeof(StageArgs),
                           hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return MPRK_EHIP;
        c->ptab_dt = dt;
    }
    if ((int64_t)nsteps * ms > (int64_t)(1 << 30)) return MPRK_EINVAL;
    const int tiles_x = (g.nx + TX - 1) / TX;
    MemberRun& mr = c->h_mr;
    std::memset(&mr, 0, sizeof mr);
    mr.stages = (const StageArgs*)(ws + c->lay.off_ptab);
    mr.nstages = (int32_t)(nsteps * ms);
    mr.ms = ms;
    mr.tiles_x = tiles_x;
    mr.tiles_z[0] = (g.nz_lower + TZ - 1) / TZ;
    mr.tiles_z[1] = (g.nz_upper + TZ - 1) / TZ;
    mr.done_base[0] = 0;
    mr.done_base[1] = tiles_x * mr.tiles_z[0];
    if (hipMemcpyAsync(ws + c->lay.off_pmember, &mr, sizeof mr, hipMemcpyHostToDevice, c->stream) !=
        hipSuccess)
        return MPRK_EHIP;
    int32_t* done = (int32_t*)(ws + c->lay.off_pdone);
    if (launch_fill_i32(done, 0, c->lay.ntiles + 1, c->stream) != hipSuccess) return MPRK_EHIP;
    PersistArgs P;
    std::memset(&P, 0, sizeof P);
    P.tiles = (const TileRef*)(ws + c->lay.off_ptiles);
    P.members = (const MemberRun*)(ws + c->lay.off_pmember);
    P.done = done;
    P.abort_flag = done + c->lay.ntiles;
    P.ntiles = c->lay.ntiles;
    P.gmax = mr.nstages;
    P.wait_ticks = c->wait_ticks;
    if (launch_persistent(P, c->pgrid, g.flux_bits == 32, c->stream) != hipSuccess) return MPRK_EHIP;
    return MPRK_OK;
}

int advance(mprk_ctx* c, double dt, int64_t nsteps)
{
    if (nsteps <= 0) return MPRK_OK;
    int rc;
    if (c->exec == MPRK_EXEC_PERSISTENT) {
        rc = run_persistent(c, dt, nsteps);
    } else {
        rc = MPRK_OK;
        for (int64_t n = 0; n < nsteps && rc == MPRK_OK; ++n) rc = step_launches(c, dt);
    }
    if (rc == MPRK_OK) c->steps += nsteps;
    return rc;
}

}  // namespace

extern "C" {

int mprk_set_exec(mprk_ctx* c, int mode)
{
    if (!c || (mode != MPRK_EXEC_LAUNCH && mode != MPRK_EXEC_PERSISTENT)) return MPRK_EINVAL;
    c->exec = mode;
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

static int run_reduce(mprk_ctx* c, mprk_stats* out)
{
    const mprk_config& g = c->cfg;
    ReduceArgs r;
    std::memset(&r, 0, sizeof r);
    r.q[0] = c->q[0];
    r.q[1] = c->q[1];
    r.nz[0] = g.nz_lower;
    r.nz[1] = g.nz_upper;
    r.nx = g.nx;
    r.inv_dx = 1.0 / g.dx;
    r.inv_dz[0] = 1.0 / g.dz_lower;
    r.inv_dz[1] = 1.0 / g.dz_upper;
    const double coef = std::max(4.0 / 3.0, g.gamma / g.prandtl);
    r.visc_coef[0] = coef * g.mu_lower * (1.0 / (g.dx * g.dx) + 1.0 / (g.dz_lower * g.dz_lower));
    r.visc_coef[1] = coef * g.mu_upper * (1.0 / (g.dx * g.dx) + 1.0 / (g.dz_upper * g.dz_upper));
    r.gamma = g.gamma;
    r.gm1 = g.gamma - 1.0;
    r.partial = (double*)(c->ws + c->lay.off_partial);
    r.final_ = (double*)(c->ws + c->lay.off_final);
    if (launch_reduce(r, c->stream) != hipSuccess) return MPRK_EHIP;
    if (hipMemcpyAsync(c->host_final, r.final_, sizeof c->host_final, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess)
        return MPRK_EHIP;
    int32_t aborted = 0;
    if (c->exec == MPRK_EXEC_PERSISTENT &&
        hipMemcpyAsync(&aborted, (int32_t*)(c->ws + c->lay.off_pdone) + c->lay.ntiles,
                       sizeof aborted, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return MPRK_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MPRK_EHIP;
    if (aborted) return MPRK_ETIMEOUT;
    mprk_stats st;
    std::memset(&st, 0, sizeof st);
    const double area[2] = {g.dx * g.dz_lower, g.dx * g.dz_upper};
    int bad = 0;
    for (int d = 0; d < 2; ++d) {
        const double* f = c->host_final + d * RED_FIELDS;
        double* tot = d == 0 ? st.totals_lower : st.totals_upper;
        for (int v = 0; v < NV; ++v) tot[v] = (f[v] + f[NV + v]) * area[d];
        (d == 0 ? st.lambda_lower : st.lambda_upper) = f[8];
        (d == 0 ? st.courant_lower : st.courant_upper) = f[9];
        (d == 0 ? st.visc_lower : st.visc_upper) = f[10];
        if (f[11] != 0.0) bad = 1;
    }
    st.steps_done = c->steps;
    st.status = bad;
    if (out) *out = st;
    return bad ? MPRK_ENONFINITE : MPRK_OK;
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

}  // extern "C"
