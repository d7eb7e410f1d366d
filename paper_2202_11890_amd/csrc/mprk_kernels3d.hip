// mprk_kernels3d.hip -- gfx950 stage kernel of the MPRK library in three
// dimensions (Appendix B, eq. ns-fv-cartesian-3d: x and y periodic, the two
// domains stacked in z and coupled through the rigid lid).
//
// Two kernels.  march_kernel3 (FP32 face fluxes, the 3D workload's precision)
// walks 32 x 8 columns of one domain upward through a z-segment, plane by
// plane, with a rolling window of staged planes in LDS.  stage_kernel3 (FP64
// face fluxes) is the brick form described next.
//
// Brick form, the 2D kernel's structure: a workgroup owns a TX x TY x TZ tile of one
// domain; each thread owns one cell (or a vertical run of cells).  The conserved state
// (5 components, 2-cell halo) and the primitives u, v, w, T (1-cell halo) are
// staged in LDS in the flux type; every face of the tile is evaluated once
// (three per cell plus the left, front and bottom edge faces), exchanged
// through LDS (aliasing the staged state), and each thread forms the
// divergence and the stage combination of its cells in FP64.  The interface
// viscous flux is computed per column in FP64 and added in the divergence.
#include "mprk_internal.h"
#include "mprk_device.h"

namespace mprk {

namespace {

#ifndef MPRK3_PATCH_X
#define MPRK3_PATCH_X 32
#endif
#ifndef MPRK3_PATCH_Y
#define MPRK3_PATCH_Y 16
#endif

template <int X, int Y, int Z, int C>
struct Shape3 {
    static constexpr int CZ = C;                        // cells per thread, stacked in z
    static constexpr int TX = X, TY = Y, TZ = Z, NT = X * Y * Z / C;
    // Tile order: x-y patches of GX x GY tiles (MPRK3_PATCH_X x MPRK3_PATCH_Y
    // cells), each walked through its z layers before the next patch.
    static constexpr int GX = MPRK3_PATCH_X / X > 0 ? MPRK3_PATCH_X / X : 1;
    static constexpr int GY = MPRK3_PATCH_Y / Y > 0 ? MPRK3_PATCH_Y / Y : 1;
    static constexpr int HX = X + 4, HY = Y + 4, HZ = Z + 4;
    static constexpr int PX = X + 2, PY = Y + 2, PZ = Z + 2;
    static constexpr int QPL = HY * HX;                 // staged state: one z-plane
    static constexpr int LDS_Q = NV3 * HZ * QPL;
    static constexpr int PPL = PY * PX;
    static constexpr int LDS_P = 4 * PZ * PPL;          // u, v, w, T
    static constexpr int EXX = Z * Y * (X + 1), EXY = Z * (Y + 1) * X, EXZ = (Z + 1) * Y * X;
    static constexpr int LDS_EX = NV3 * (EXX + EXY + EXZ);
    static_assert(Z % C == 0 && NT % 64 == 0 && NT <= 1024, "tile shape");
    static_assert(LDS_EX <= LDS_Q + LDS_P, "flux exchange must fit in the staged state");
    template <class FT>
    static constexpr int lds_bytes() { return (LDS_Q + LDS_P) * (int)sizeof(FT) + 3 * X * Y * 8; }
};

using T64 = Shape3<16, 4, 4, 1>;            // FP64 fluxes: 73.5 KB LDS, 256 threads

// Brick tile per flux type (FP32 fluxes run the marching kernel instead).
template <class FT> struct TileOf;
template <> struct TileOf<double> { using S = T64; };

template <class FT>
struct Lds3 {
    FT* q;        // [5][HZ][HY][HX]
    FT* p;        // [4][PZ][PY][PX]
    double* gf;   // [3][TY*TX]: interface flux (x-, y-momentum, energy) per column
};

template <class S>
__device__ __forceinline__ int q3(int v, int z, int y, int x)
{
    return ((v * S::HZ + z + 2) * S::HY + y + 2) * S::HX + x + 2;
}
template <class S>
__device__ __forceinline__ int p3(int f, int z, int y, int x)
{
    return ((f * S::PZ + z + 1) * S::PY + y + 1) * S::PX + x + 1;
}

enum : int { F3_INTERIOR = 0, F3_TOP = 1, F3_BOTTOM = 2 };

template <class FT>
__device__ __forceinline__ void prim3(const FT* c, FT gamma, FT gm1, FT& u, FT& v, FT& w, FT& T)
{
    // Every tile that stages a cell computes its primitives: contraction off
    // and the fused operations written out, so all obtain the same bits.
#pragma clang fp contract(off)
    const FT ir = Fm<FT>::rcp(c[0]);
    u = c[1] * ir;
    v = c[2] * ir;
    w = c[3] * ir;
    const FT p = gm1 * fma(FT(-0.5), fma(c[1], u, fma(c[2], v, c[3] * w)), c[4]);
    T = gamma * p * ir;
}

// FP64 u, v, T of a cell next to the interface; contraction off and the same
// code in the tiles on both sides, so both obtain the same bits.
__device__ __forceinline__ void interface_cell3(const double* c, double gamma, double gm1, double& u,
                                                double& v, double& T)
{
#pragma clang fp contract(off)
    const double ir = rcp_nr(c[0]);
    u = c[1] * ir;
    v = c[2] * ir;
    const double w = c[3] * ir;
    const double p = gm1 * (c[4] - 0.5 * (c[1] * u + c[2] * v + c[3] * w));
    T = gamma * p * ir;
}

// Interface viscous flux in +z (Appendix B, eq. bulk-flux with b_v = b_u):
// (0, sigma_xz, sigma_yz, 0, u_w sigma_xz + v_w sigma_yz - Pi_z).
__device__ __forceinline__ void interface_flux3(const StageArgs& A, double u1, double v1, double T1,
                                                double u2, double v2, double T2, double* f)
{
#pragma clang fp contract(off)
    const double sx = A.bu * (u2 - u1);
    const double sy = A.bu * (v2 - v1);
    const double pi = -A.bT * (T2 - T1);
    const double uw = u1 + sx * A.half_dz1_mu1;
    const double vw = v1 + sy * A.half_dz1_mu1;
    f[0] = sx;
    f[1] = sy;
    f[2] = uw * sx + vw * sy - pi;
}

// Numerical flux through the face between tile cell (x, y, z) and its +dir
// neighbour, in the components (rho, rho u, rho v, rho w, rho E).  Kinds as
// in 2D (F3_TOP / F3_BOTTOM: mirror faces in z, no viscous part).
template <class FT, int dir, class S>
__device__ __forceinline__ void face3(const StageArgs& A, const DomainArgs& D, const Lds3<FT>& L, int x,
                                      int y, int z, int kind, FT F[NV3])
{
#pragma clang fp contract(off)
    const FT gamma = arg_ft<FT>(A.gamma, A.gamma_f), gm1 = arg_ft<FT>(A.gm1, A.gm1_f);
    const FT h = FT(0.5), q4 = FT(0.25);
    constexpr int sn = dir == 0 ? 1 : (dir == 1 ? S::HX : S::QPL);
    constexpr int t1 = (dir + 1) % 3, t2 = (dir + 2) % 3;   // tangential directions
    constexpr int plane = S::HZ * S::QPL;
    // components in the face frame: rho, normal, tangential 1, tangential 2, energy
    constexpr int comp[NV3] = {0, 1 + dir, 1 + t1, 1 + t2, 4};

    FT qL[NV3], qR[NV3];
    const int base = q3<S>(0, z, y, x);
#pragma unroll
    for (int k = 0; k < NV3; ++k) {
        const FT* s = L.q + comp[k] * plane + base;
        const FT qm = s[-sn], q0 = s[0], q1 = s[sn], q2 = s[2 * sn];
        qL[k] = fma(q4, q1 - qm, q0);
        qR[k] = fma(-q4, q2 - q0, q1);
    }
    if (kind == F3_TOP) {
        qR[0] = qL[0]; qR[1] = -qL[1]; qR[2] = qL[2]; qR[3] = qL[3]; qR[4] = qL[4];
    } else if (kind == F3_BOTTOM) {
        qL[0] = qR[0]; qL[1] = -qR[1]; qL[2] = qR[2]; qL[3] = qR[3]; qL[4] = qR[4];
    }
    const FT yL = Fm<FT>::rsqrt(qL[0]), yR = Fm<FT>::rsqrt(qR[0]);
    const FT rL = yL * yL, rR = yR * yR;
    const FT sL = qL[0] * yL, sR = qR[0] * yR;
    const FT unL = qL[1] * rL, a1L = qL[2] * rL, a2L = qL[3] * rL;
    const FT unR = qR[1] * rR, a1R = qR[2] * rR, a2R = qR[3] * rR;
    const FT pL = gm1 * fma(-h, fma(qL[1], unL, fma(qL[2], a1L, qL[3] * a2L)), qL[4]);
    const FT pR = gm1 * fma(-h, fma(qR[1], unR, fma(qR[2], a1R, qR[3] * a2R)), qR[4]);
    const FT aL = Fm<FT>::ws_sqrt(gamma * pL * rL);
    const FT aR = Fm<FT>::ws_sqrt(gamma * pR * rR);
    const FT iw = Fm<FT>::ws_rcp(sL + sR);
    const FT unr = fma(sL, unL, sR * unR) * iw;
    const FT a1r = fma(sL, a1L, sR * a1R) * iw;
    const FT a2r = fma(sL, a2L, sR * a2R) * iw;
    const FT HL = (qL[4] + pL) * rL, HR = (qR[4] + pR) * rR;
    const FT Hr = fma(sL, HL, sR * HR) * iw;
    const FT ar = Fm<FT>::ws_sqrt(gm1 * fma(-h, fma(unr, unr, fma(a1r, a1r, a2r * a2r)), Hr));
    const FT lam = fmax(fmax(fabs(unL) + aL, fabs(unR) + aR), fabs(unr) + ar);
    FT Fn[NV3];
    if (kind != F3_INTERIOR) {
        // Against its mirror image: (0, rho u_n^2 + p +- lambda rho u_n, 0, 0, 0).
        Fn[0] = FT(0);
        Fn[1] = (kind == F3_TOP) ? fma(lam, qL[1], fma(qL[1], unL, pL)) : fma(-lam, qR[1], fma(qR[1], unR, pR));
        Fn[2] = FT(0);
        Fn[3] = FT(0);
        Fn[4] = FT(0);
    } else {
        const FT hl = h * lam;
        Fn[0] = fma(-hl, qR[0] - qL[0], h * (qL[1] + qR[1]));
        Fn[1] = fma(-hl, qR[1] - qL[1], h * (fma(qL[1], unL, qR[1] * unR) + (pL + pR)));
        Fn[2] = fma(-hl, qR[2] - qL[2], h * fma(qL[2], unL, qR[2] * unR));
        Fn[3] = fma(-hl, qR[3] - qL[3], h * fma(qL[3], unL, qR[3] * unR));
        Fn[4] = fma(-hl, qR[4] - qL[4], h * fma(qL[4] + pL, unL, (qR[4] + pR) * unR));

        // Viscous part (Appendix B): common velocity, normal derivatives by
        // finite difference, tangential ones by averaging the cell gradients.
        constexpr int pn = dir == 0 ? 1 : (dir == 1 ? S::PX : S::PPL);
        constexpr int ps[3] = {1, S::PX, S::PPL};
        constexpr int pp = S::PZ * S::PPL;
        const int pb = p3<S>(0, z, y, x);
        const FT inv_h[3] = {arg_ft<FT>(A.inv_dx, A.inv_dx_f), arg_ft<FT>(A.inv_dy, A.inv_dy_f),
                             arg_ft<FT>(D.inv_dz, D.inv_dz_f)};
        // g[c][d]: d u_c / d x_d at the face, c, d in (x, y, z)
        FT g[3][3], uh[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const FT* U = L.p + c * pp + pb;
            uh[c] = h * (U[0] + U[pn]);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (d == dir) {
                    g[c][d] = (U[pn] - U[0]) * inv_h[d];
                } else {
                    const int st = ps[d];
                    g[c][d] = ((U[st] - U[-st]) + (U[pn + st] - U[pn - st])) * (q4 * inv_h[d]);
                }
            }
        }
        const FT* Tt = L.p + 3 * pp + pb;
        const FT Tn = (Tt[pn] - Tt[0]) * inv_h[dir];
        const FT mu = arg_ft<FT>(D.mu, D.mu_f);
        FT sg[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            sg[c] = (c == dir) ? mu * fma(FT(4.0 / 3.0), g[dir][dir], FT(-2.0 / 3.0) * (g[t1][t1] + g[t2][t2]))
                               : mu * (g[dir][c] + g[c][dir]);
        const FT en = fma(uh[0], sg[0], fma(uh[1], sg[1], fma(uh[2], sg[2], arg_ft<FT>(D.kappa, D.kappa_f) * Tn)));
        Fn[1] = Fn[1] - sg[dir];
        Fn[2] = Fn[2] - sg[t1];
        Fn[3] = Fn[3] - sg[t2];
        Fn[4] = Fn[4] - en;
    }
    // back to (rho, rho u, rho v, rho w, rho E)
    F[0] = Fn[0];
    F[1 + dir] = Fn[1];
    F[1 + t1] = Fn[2];
    F[1 + t2] = Fn[3];
    F[4] = Fn[4];
}

// Tile t of a domain's launch range -> tile coordinates.  The x-y plane is
// cut into strips of GY tile rows and each strip into patches of GX tile
// columns (the last strip and patch may be narrower); a patch is walked layer
// by layer in z, x fastest, before the next patch starts.  Workgroups that run
// at the same time on one XCD (which owns a contiguous range of t) then form a
// compact block whose x-y halos overlap, and the layers below a block were
// staged just before it, so the halo re-reads of the 2-cell stencil mostly
// hit that XCD's L2 instead of HBM.  The map is a bijection onto
// [0, tiles_x) x [0, tiles_y) x [0, tiles_z).
template <class S>
__device__ __forceinline__ void tile_coords3(int t, int tiles_x, int tiles_y, int tiles_z, int& tx,
                                             int& ty, int& tz)
{
    const int strip = S::GY * tiles_x * tiles_z;
    const int j = t / strip;
    int r = t - j * strip;
    const int wy = min(S::GY, tiles_y - j * S::GY);
    const int patch = S::GX * wy * tiles_z;
    const int i = r / patch;
    r -= i * patch;
    const int wx = min(S::GX, tiles_x - i * S::GX);
    tz = r / (wx * wy);
    r -= tz * (wx * wy);
    ty = j * S::GY + r / wx;
    tx = i * S::GX + r % wx;
}

template <int DOM, class FT>
__device__ __forceinline__ void stage_tile3(const StageArgs& A, int tile, char* smem)
{
    using S = typename TileOf<FT>::S;
    constexpr int TX = S::TX, TY = S::TY, TZ = S::TZ, NT = S::NT;
    constexpr int HX = S::HX, HY = S::HY, HZ = S::HZ, PX = S::PX, PY = S::PY, PZ = S::PZ;
    const DomainArgs& D = A.d[DOM];
    const DomainArgs& O = A.d[1 - DOM];
    const int tid = threadIdx.x;
    const int nx = A.nx, ny = A.ny, nz = D.nz;
    int tx, ty, tz;
    tile_coords3<S>(tile, D.tiles_x, D.tiles_y, D.tiles_z, tx, ty, tz);
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = (D.row_lo / TZ + tz) * TZ;
    const int vs = max(z0, D.row_lo) - z0;
    const int ve = min(z0 + TZ, D.row_hi) - z0;
    const int ncx = min(TX, nx - x0), ncy = min(TY, ny - y0);
    const size_t rowsz = (size_t)ny * nx;

    Lds3<FT> L;
    L.q = (FT*)smem;
    L.p = L.q + S::LDS_Q;
    L.gf = (double*)(smem + (S::LDS_Q + S::LDS_P) * sizeof(FT));
    FT* ex_x = L.q;                       // [5][TZ][TY][TX+1]
    FT* ex_y = ex_x + NV3 * S::EXX;       // [5][TZ][TY+1][TX]
    FT* ex_z = ex_y + NV3 * S::EXY;       // [5][TZ+1][TY][TX]

    const bool has_gamma = (DOM == 0) ? (D.gamma_top && z0 + ve == nz) : (D.gamma_bot && z0 + vs == 0);

    constexpr int CZ = S::CZ;
    const int cx = tid % TX;
    const int cy = (tid / TX) % TY;
    const int r0 = CZ * (tid / (TX * TY));
    const bool inxy = cx < ncx && cy < ncy;
    bool okc[CZ];
#pragma unroll
    for (int hh = 0; hh < CZ; ++hh) okc[hh] = inxy && r0 + hh >= vs && r0 + hh < ve;

    // Raised issue priority while the tile's global loads go out (as in 2D;
    // 1% per step on the 256 x 256 x 128 workload).
    __builtin_amdgcn_s_setprio(2);
    // ---- stage the state (x, y periodic; mirror planes beyond the domain;
    // retained slow planes at substeps 2..m).  Each loader thread owns one
    // (x, y) position of the staged tile and every LOAD_RG-th plane, so the
    // periodic wrap and the column offset are computed once (against one
    // decomposition of the cell index per staged cell: 4% per step with FP64
    // fluxes, 1% with FP32); the global loads of LOAD_B planes are issued
    // before any is stored.
    constexpr int NCELL = HZ * HY * HX;
    constexpr int NPC = PZ * PY * PX;
    constexpr int PXY = HY * HX;
    constexpr int LOAD_RG = NT / PXY;
    static_assert(LOAD_RG >= 1, "loader needs a full plane of threads");
    constexpr int LOAD_PL = (HZ + LOAD_RG - 1) / LOAD_RG;   // planes per loader thread
    // Planes whose loads are issued together: measured best at 2 for the
    // FP32-flux tile (4 planes per thread) and 4 for the FP64-flux tile (8).
    constexpr int LOAD_BMAX = sizeof(FT) == 8 ? 4 : 2;
    constexpr int LOAD_B = LOAD_PL < LOAD_BMAX ? LOAD_PL : LOAD_BMAX;
    if (tid < LOAD_RG * PXY) {
        const int pos = tid % PXY, rg = tid / PXY;
        const int yy = pos / HX, xx = pos - yy * HX;
        const bool near = nx > TX && ny > TY;
        const int col = near ? wrap1(x0 + xx - 2, nx) : wrapx(x0 + xx - 2, nx);
        const int rowy = near ? wrap1(y0 + yy - 2, ny) : wrapx(y0 + yy - 2, ny);
        const size_t cofs = (size_t)rowy * nx + col;
        for (int k0 = 0; k0 < LOAD_PL; k0 += LOAD_B) {
            double val[LOAD_B][NV3];
            bool neg[LOAD_B];
#pragma unroll
            for (int u = 0; u < LOAD_B; ++u) {
                const int zz = rg + LOAD_RG * (k0 + u);
                neg[u] = false;
                if (k0 + u < LOAD_PL && zz < HZ) {
                    int pl = z0 + zz - 2;
                    if (pl < 0) { pl = 0; neg[u] = true; }
                    else if (pl >= nz) { pl = nz - 1; neg[u] = true; }
                    const double* src;
                    size_t vstride;
                    if (D.use_ret && (pl < D.b_lo || pl >= D.b_hi)) {
                        int rr = pl - D.ret_lo;
                        rr = rr < 0 ? 0 : (rr > 1 ? 1 : rr);
                        src = D.ret_in + (size_t)rr * rowsz + cofs;
                        vstride = 2 * rowsz;
                    } else {
                        src = D.qin + (size_t)pl * rowsz + cofs;
                        vstride = (size_t)nz * rowsz;
                    }
#pragma unroll
                    for (int v = 0; v < NV3; ++v) val[u][v] = src[v * vstride];
                }
            }
#pragma unroll
            for (int u = 0; u < LOAD_B; ++u) {
                const int zz = rg + LOAD_RG * (k0 + u);
                if (k0 + u < LOAD_PL && zz < HZ) {
                    const int idx = zz * PXY + pos;
                    FT c[NV3];
#pragma unroll
                    for (int v = 0; v < NV3; ++v) {
                        c[v] = FT((v == 3 && neg[u]) ? -val[u][v] : val[u][v]);
                        L.q[v * NCELL + idx] = c[v];
                    }
                    // Primitives of the tile and its 1-cell ring, from the
                    // same staged values (primitive cell (zz-1, yy-1, xx-1)).
                    if (xx >= 1 && xx <= HX - 2 && yy >= 1 && yy <= HY - 2 && zz >= 1 && zz <= HZ - 2) {
                        FT pu, pv, pw, pT;
                        prim3<FT>(c, arg_ft<FT>(A.gamma, A.gamma_f), arg_ft<FT>(A.gm1, A.gm1_f), pu, pv, pw,
                              pT);
                        const int pi = ((zz - 1) * PY + yy - 1) * PX + xx - 1;
                        L.p[pi] = pu;
                        L.p[NPC + pi] = pv;
                        L.p[2 * NPC + pi] = pw;
                        L.p[3 * NPC + pi] = pT;
                    }
                }
            }
        }
    }
    // Interface flux per column, FP64 from the FP64 cells next to the lid.
    if (has_gamma) {
        for (int c = tid; c < TX * TY; c += NT) {
            const int xx = c % TX, yy = c / TX;
            const bool near = nx > TX && ny > TY;
            const int col = near ? wrap1(x0 + xx, nx) : wrapx(x0 + xx, nx);
            const int rowy = near ? wrap1(y0 + yy, ny) : wrapx(y0 + yy, ny);
            const int own = (DOM == 0) ? nz - 1 : 0;
            const int oth = (DOM == 0) ? 0 : O.nz - 1;
            const size_t po = (size_t)nz * rowsz, pq = (size_t)O.nz * rowsz;
            const double* a = D.qin + (size_t)own * rowsz + (size_t)rowy * nx + col;
            const double* b = O.qin + (size_t)oth * rowsz + (size_t)rowy * nx + col;
            double ca[NV3], cb[NV3];
#pragma unroll
            for (int v = 0; v < NV3; ++v) { ca[v] = a[v * po]; cb[v] = b[v * pq]; }
            double ua, va, Ta, ub, vb, Tb, f[3];
            interface_cell3(ca, A.gamma, A.gm1, ua, va, Ta);
            interface_cell3(cb, A.gamma, A.gm1, ub, vb, Tb);
            if (DOM == 0) interface_flux3(A, ua, va, Ta, ub, vb, Tb, f);
            else interface_flux3(A, ub, vb, Tb, ua, va, Ta, f);
            L.gf[c] = f[0];
            L.gf[TX * TY + c] = f[1];
            L.gf[2 * TX * TY + c] = f[2];
        }
    }
    __syncthreads();

    __builtin_amdgcn_s_setprio(0);

    // ---- faces: x+, y+, z+ of the thread's cells, then the edge faces
    // (x left of column 0, y in front of row 0, z below the first computed
    // plane), all kept in registers or written after the barrier.
    FT F[3 * CZ][NV3];
#pragma unroll
    for (int hh = 0; hh < CZ; ++hh) {
        if (!okc[hh]) continue;
        const int kz = (z0 + r0 + hh == nz - 1) ? F3_TOP : F3_INTERIOR;
        face3<FT, 0, S>(A, D, L, cx, cy, r0 + hh, F3_INTERIOR, F[3 * hh]);
        face3<FT, 1, S>(A, D, L, cx, cy, r0 + hh, F3_INTERIOR, F[3 * hh + 1]);
        face3<FT, 2, S>(A, D, L, cx, cy, r0 + hh, kz, F[3 * hh + 2]);
    }
    // Edge faces: ne_x = TY*TZ (x = -1), ne_y = TX*TZ (y = -1), ne_z = TX*TY
    // (below vs).  Each direction's range of edge indices starts at a wave
    // boundary, so that no wave runs the face code of two directions.
    constexpr int NEX = TY * TZ, NEY = TX * TZ, NEZ = TX * TY;
    constexpr int OEY = (NEX + 63) / 64 * 64, OEZ = OEY + (NEY + 63) / 64 * 64, NE = OEZ + NEZ;
    constexpr int EPT = (NE + NT - 1) / NT;
    FT E[EPT][NV3];
    int ekind[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + u * NT;
        ekind[u] = -1;
        if (e < NEX) {
            const int yy = e % TY, zz = e / TY;
            if (yy < ncy && zz >= vs && zz < ve) {
                face3<FT, 0, S>(A, D, L, -1, yy, zz, F3_INTERIOR, E[u]);
                ekind[u] = 0;
            }
        } else if (e >= OEY && e < OEY + NEY) {
            const int f = e - OEY, xx = f % TX, zz = f / TX;
            if (xx < ncx && zz >= vs && zz < ve) {
                face3<FT, 1, S>(A, D, L, xx, -1, zz, F3_INTERIOR, E[u]);
                ekind[u] = 1;
            }
        } else if (e >= OEZ && e < NE) {
            const int f = e - OEZ, xx = f % TX, yy = f / TX;
            if (xx < ncx && yy < ncy) {
                const int kind = (z0 + vs == 0) ? F3_BOTTOM : F3_INTERIOR;
                face3<FT, 2, S>(A, D, L, xx, yy, vs - 1, kind, E[u]);
                ekind[u] = 2;
            }
        }
    }

    __builtin_amdgcn_s_setprio(2);
    // FP64 pointwise reads for the combination (the stage value itself when
    // the fluxes are FP32; the substep base U).
    const int col = x0 + cx, rowy = y0 + cy;
    const size_t plane = (size_t)nz * rowsz;
    const size_t nbx = (size_t)(D.b_hi - D.b_lo) * rowsz;
    double qc[CZ][NV3], Ub[CZ][NV3];
#pragma unroll
    for (int hh = 0; hh < CZ; ++hh) {
        const int row = z0 + r0 + hh;
        const bool ok = okc[hh];
        const bool inb = (row >= D.b_lo && row < D.b_hi);
        const Combine cb = pick_combine(D.buf, D.main, inb);
        const size_t id = (size_t)row * rowsz + (size_t)rowy * nx + col;
#pragma unroll
        for (int v = 0; v < NV3; ++v) {
            Ub[hh][v] = 0.0;
            qc[hh][v] = sizeof(FT) == 8 ? (double)L.q[q3<S>(v, r0 + hh, cy, cx)] : 0.0;
        }
        if (ok && sizeof(FT) != 8) {
#pragma unroll
            for (int v = 0; v < NV3; ++v) qc[hh][v] = D.qin[v * plane + id];
        }
        if (ok && cb.mode != MODE_RHS && cb.alpha != 0.0) {
#pragma unroll
            for (int v = 0; v < NV3; ++v) Ub[hh][v] = D.base[v * plane + id];
        }
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();   // all LDS reads of the staged state are done

    auto put = [&](int d, int xx, int yy, int zz, const FT* f) {
        FT* e;
        int st;
        if (d == 0) { e = ex_x + (zz * TY + yy) * (TX + 1) + xx + 1; st = S::EXX; }
        else if (d == 1) { e = ex_y + (zz * (TY + 1) + yy + 1) * TX + xx; st = S::EXY; }
        else { e = ex_z + ((zz + 1) * TY + yy) * TX + xx; st = S::EXZ; }
#pragma unroll
        for (int v = 0; v < NV3; ++v) e[v * st] = f[v];
    };
#pragma unroll
    for (int hh = 0; hh < CZ; ++hh) {
        if (!okc[hh]) continue;
        put(0, cx, cy, r0 + hh, F[3 * hh]);
        put(1, cx, cy, r0 + hh, F[3 * hh + 1]);
        put(2, cx, cy, r0 + hh, F[3 * hh + 2]);
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + u * NT;
        if (ekind[u] == 0) put(0, -1, e % TY, e / TY, E[u]);
        else if (ekind[u] == 1) { const int f = e - OEY; put(1, f % TX, -1, f / TX, E[u]); }
        else if (ekind[u] == 2) { const int f = e - OEZ; put(2, f % TX, f / TX, vs - 1, E[u]); }
    }
    __syncthreads();

    // ---- divergence (FP64), interface flux, source, stage combination
    const double inv_dx = A.inv_dx, inv_dy = A.inv_dy, inv_dz = D.inv_dz;
#pragma unroll
    for (int hh = 0; hh < CZ; ++hh) {
        if (!okc[hh]) continue;
        const int zz = r0 + hh;
        const int row = z0 + zz;
        double R[NV3];
#pragma unroll
        for (int v = 0; v < NV3; ++v) {
            const FT* fx = ex_x + v * S::EXX + (zz * TY + cy) * (TX + 1) + cx;
            const FT* fy = ex_y + v * S::EXY + (zz * (TY + 1) + cy) * TX + cx;
            const FT* fz = ex_z + v * S::EXZ + (zz * TY + cy) * TX + cx;
            // The +x, +y and +z faces are this thread's own (still in
            // registers); the other three come from the exchange.
            R[v] = -((double)F[3 * hh][v] - (double)fx[0]) * inv_dx -
                   ((double)F[3 * hh + 1][v] - (double)fy[0]) * inv_dy -
                   ((double)F[3 * hh + 2][v] - (double)fz[0]) * inv_dz;
        }
        const int gc = cy * TX + cx;
        if (DOM == 0 && D.gamma_top && row == nz - 1) {
            R[1] += L.gf[gc] * inv_dz;
            R[2] += L.gf[TX * TY + gc] * inv_dz;
            R[4] += L.gf[2 * TX * TY + gc] * inv_dz;
        }
        if (DOM == 1 && D.gamma_bot && row == 0) {
            R[1] -= L.gf[gc] * inv_dz;
            R[2] -= L.gf[TX * TY + gc] * inv_dz;
            R[4] -= L.gf[2 * TX * TY + gc] * inv_dz;
        }
        R[3] += qc[hh][0] * A.gravity;
        R[4] += qc[hh][3] * A.gravity;

        const bool inb = (row >= D.b_lo && row < D.b_hi);
        const Combine cb = pick_combine(D.buf, D.main, inb);
        const size_t id = (size_t)row * rowsz + (size_t)rowy * nx + col;
        if (cb.mode == MODE_RHS) {
#pragma unroll
            for (int v = 0; v < NV3; ++v) st_dev(A.dev_stores != 0, &D.out[v * plane + id], R[v]);
        } else if (cb.alpha == 0.0) {
#pragma unroll
            for (int v = 0; v < NV3; ++v) st_dev(A.dev_stores != 0, &D.out[v * plane + id], qc[hh][v] + cb.bh * R[v]);
        } else {
            double inc[NV3];
#pragma unroll
            for (int v = 0; v < NV3; ++v) inc[v] = cb.beta * (qc[hh][v] - Ub[hh][v]) + cb.bh * R[v];
            if (cb.mode == MODE_STAGE) {
#pragma unroll
                for (int v = 0; v < NV3; ++v) st_dev(A.dev_stores != 0, &D.out[v * plane + id], Ub[hh][v] + inc[v]);
            } else {
                const size_t ia = (size_t)(row - D.b_lo) * rowsz + (size_t)rowy * nx + col;
                if (cb.mode == MODE_ACC_FIRST) {
#pragma unroll
                    for (int v = 0; v < NV3; ++v) st_dev(A.dev_stores != 0, &D.acc[v * nbx + ia], inc[v]);
                } else if (cb.mode == MODE_ACC_ADD) {
#pragma unroll
                    for (int v = 0; v < NV3; ++v) st_dev(A.dev_stores != 0, &D.acc[v * nbx + ia], D.acc[v * nbx + ia] + inc[v]);
                } else {
#pragma unroll
                    for (int v = 0; v < NV3; ++v)
                        st_dev(A.dev_stores != 0, &D.out[v * plane + id], Ub[hh][v] + (D.acc[v * nbx + ia] + inc[v]) * A.inv_m);
                }
            }
        }
        if (D.ret_out && row >= D.ret_lo && row < D.ret_lo + 2) {
#pragma unroll
            for (int v = 0; v < NV3; ++v)
                st_dev(A.dev_stores != 0, &D.ret_out[(size_t)(v * 2 + row - D.ret_lo) * rowsz + (size_t)rowy * nx + col], qc[hh][v]);
        }
    }
}

template <class FT>
__global__ __launch_bounds__(TileOf<FT>::S::NT) void stage_kernel3(const StageArgs A)
{
    using S = typename TileOf<FT>::S;
    __shared__ __align__(16) char smem[S::template lds_bytes<FT>()];
    const int b = xcd_contiguous(blockIdx.x, A.nblocks);
    const int n0 = A.d[A.first].ntiles;
    const int dom = (b < n0) ? A.first : 1 - A.first;
    const int t = (b < n0) ? b : b - n0;
    if (dom == 0) stage_tile3<0, FT>(A, t, smem);
    else stage_tile3<1, FT>(A, t, smem);
}

// ---------------------------------------------------------------------------
// z-marching stage kernel (used with FP32 face fluxes).  A workgroup owns a
// TX x TY block of columns and one segment of LZ planes of a domain and walks
// the segment upward, one plane per step.  LDS holds a two-plane ring of the
// staged state (2-cell x-y halo), a three-plane ring of the primitives
// u, v, w, T (1-cell halo) and the x-y flux exchange; each thread keeps its
// own column's state at planes z-1 .. z+2 in registers.  Per plane: the x and
// y faces of the plane come from the staged plane; the z-face above it from
// the column registers; the z-face below it is the one computed at the
// previous plane (only a segment's first plane computes its lower face).  A
// plane is staged once per segment (the brick kernel staged each cell of a
// 2-plane z-halo for every 4-plane tile), and the next plane's global loads
// are in flight while the current one is computed.  A thread stages its own
// cell itself and keeps the low word of its FP64 value, so that the FP64
// stage value of the combination is rebuilt from the FP32 copy in LDS rather
// than read from memory a second time.
template <int X, int Y, int L>
struct MShape {
    static constexpr int TX = X, TY = Y, LZ = L, NT = X * Y;
    static constexpr int HX = X + 4, HY = Y + 4, QPL = HX * HY;   // staged plane, 2-cell halo
    static constexpr int PX = X + 2, PY = Y + 2, PPL = PX * PY;   // primitive plane, 1-cell halo
    static constexpr int EXX = Y * (X + 1), EXY = (Y + 1) * X;    // x-y flux exchange
    static constexpr int NPOS = (QPL + NT - 1) / NT;              // staged positions per thread
    static constexpr int LDS_Q = 2 * NV3 * QPL;
    static constexpr int LDS_P = 3 * 4 * PPL;
    static constexpr int LDS_X = NV3 * (EXX + EXY);
    static_assert(NT % 64 == 0 && NT <= 1024 && NT >= 64 + X && Y <= 64, "marching tile shape");
    template <class FT>
    static constexpr int lds_bytes() { return (LDS_Q + LDS_P + LDS_X) * (int)sizeof(FT) + 3 * X * Y * 8; }
};

#ifndef MPRK3_MARCH_TX
#define MPRK3_MARCH_TX 32
#endif
#ifndef MPRK3_MARCH_TY
#define MPRK3_MARCH_TY 8
#endif
#ifndef MPRK3_MARCH_LZ
#define MPRK3_MARCH_LZ 16
#endif
#ifndef MPRK3_MARCH_WAVES
#define MPRK3_MARCH_WAVES 3
#endif
using M32 = MShape<MPRK3_MARCH_TX, MPRK3_MARCH_TY, MPRK3_MARCH_LZ>;

// Low word of an FP64 value x whose FP32 copy (round to nearest) is hi.  When
// hi is zero but x is not, the word is 1, which no zero has, so that
// join_low declines it.
__device__ __forceinline__ uint32_t low_word(double x, float hi)
{
    const uint32_t w = (uint32_t)(unsigned long long)__double_as_longlong(x);
    return (hi == 0.0f && x != 0.0) ? 1u : w;
}

// The FP64 value from its FP32 round-to-nearest copy hi and its low word lo.
// The value truncated to FP32 carries the FP64 value's sign, exponent and top
// 20 significand bits, i.e. its high word.  That truncation is hi itself when
// rounding went toward zero and hi one unit toward zero otherwise; the two
// cases differ in the truncation's last significand bit, which is bit 29 of
// lo, so comparing it with hi's last bit tells them apart.  Exact when |hi|
// lies strictly above the smallest normal FP32 number and below infinity (the
// truncation is then a normal number), and for signed zeros; ok is false
// otherwise (tiny, subnormal, overflowing and non-finite values, and |hi| equal
// to the smallest normal), and the caller reads the value from memory.
__device__ __forceinline__ double join_low(float hi, uint32_t lo, bool& ok)
{
    const uint32_t hb = __float_as_uint(hi);
    const uint32_t tb = hb - (((lo >> 29) ^ hb) & 1u);
    const uint32_t hm = hb & 0x7fffffffu;
    ok = (hm - 0x00800001u < 0x7f800000u - 0x00800001u) || ((hm | lo) == 0u);
    const unsigned long long hw =
        (unsigned long long)__double_as_longlong((double)__uint_as_float(tb)) & 0xffffffff00000000ull;
    return __longlong_as_double((long long)(hw | lo));
}

// Inviscid LLF flux of a face in its normal frame from the reconstructed
// states qL, qR (face frame: rho, normal, tangential 1, tangential 2,
// energy); mirror kinds as in face3, whose arithmetic this repeats, so a face
// evaluated by two tiles obtains the same bits from the same inputs.
template <class FT>
__device__ __forceinline__ void llf3n(const StageArgs& A, FT qL[NV3], FT qR[NV3], int kind, FT Fn[NV3])
{
#pragma clang fp contract(off)
    const FT gamma = arg_ft<FT>(A.gamma, A.gamma_f), gm1 = arg_ft<FT>(A.gm1, A.gm1_f);
    const FT h = FT(0.5);
    if (kind == F3_TOP) {
        qR[0] = qL[0]; qR[1] = -qL[1]; qR[2] = qL[2]; qR[3] = qL[3]; qR[4] = qL[4];
    } else if (kind == F3_BOTTOM) {
        qL[0] = qR[0]; qL[1] = -qR[1]; qL[2] = qR[2]; qL[3] = qR[3]; qL[4] = qR[4];
    }
    const FT yL = Fm<FT>::rsqrt(qL[0]), yR = Fm<FT>::rsqrt(qR[0]);
    const FT rL = yL * yL, rR = yR * yR;
    const FT sL = qL[0] * yL, sR = qR[0] * yR;
    const FT unL = qL[1] * rL, a1L = qL[2] * rL, a2L = qL[3] * rL;
    const FT unR = qR[1] * rR, a1R = qR[2] * rR, a2R = qR[3] * rR;
    const FT pL = gm1 * fma(-h, fma(qL[1], unL, fma(qL[2], a1L, qL[3] * a2L)), qL[4]);
    const FT pR = gm1 * fma(-h, fma(qR[1], unR, fma(qR[2], a1R, qR[3] * a2R)), qR[4]);
    const FT aL = Fm<FT>::ws_sqrt(gamma * pL * rL);
    const FT aR = Fm<FT>::ws_sqrt(gamma * pR * rR);
    const FT iw = Fm<FT>::ws_rcp(sL + sR);
    const FT unr = fma(sL, unL, sR * unR) * iw;
    const FT a1r = fma(sL, a1L, sR * a1R) * iw;
    const FT a2r = fma(sL, a2L, sR * a2R) * iw;
    const FT HL = (qL[4] + pL) * rL, HR = (qR[4] + pR) * rR;
    const FT Hr = fma(sL, HL, sR * HR) * iw;
    const FT ar = Fm<FT>::ws_sqrt(gm1 * fma(-h, fma(unr, unr, fma(a1r, a1r, a2r * a2r)), Hr));
    const FT lam = fmax(fmax(fabs(unL) + aL, fabs(unR) + aR), fabs(unr) + ar);
    if (kind != F3_INTERIOR) {
        Fn[0] = FT(0);
        Fn[1] = (kind == F3_TOP) ? fma(lam, qL[1], fma(qL[1], unL, pL)) : fma(-lam, qR[1], fma(qR[1], unR, pR));
        Fn[2] = FT(0);
        Fn[3] = FT(0);
        Fn[4] = FT(0);
        return;
    }
    const FT hl = h * lam;
    Fn[0] = fma(-hl, qR[0] - qL[0], h * (qL[1] + qR[1]));
    Fn[1] = fma(-hl, qR[1] - qL[1], h * (fma(qL[1], unL, qR[1] * unR) + (pL + pR)));
    Fn[2] = fma(-hl, qR[2] - qL[2], h * fma(qL[2], unL, qR[2] * unR));
    Fn[3] = fma(-hl, qR[3] - qL[3], h * fma(qL[3], unL, qR[3] * unR));
    Fn[4] = fma(-hl, qR[4] - qL[4], h * fma(qL[4] + pL, unL, (qR[4] + pR) * unR));
}

// Viscous part of an interior face (Appendix B: common velocity, normal
// derivatives by finite difference, tangential ones by averaging the cell
// gradients), subtracted from the inviscid flux Fn in the face frame.
template <class FT, int dir>
__device__ __forceinline__ void visc3n(const DomainArgs& D, const FT uh[3], const FT g[3][3], FT Tn, FT Fn[NV3])
{
#pragma clang fp contract(off)
    constexpr int t1 = (dir + 1) % 3, t2 = (dir + 2) % 3;
    const FT mu = arg_ft<FT>(D.mu, D.mu_f);
    FT sg[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        sg[c] = (c == dir) ? mu * fma(FT(4.0 / 3.0), g[dir][dir], FT(-2.0 / 3.0) * (g[t1][t1] + g[t2][t2]))
                           : mu * (g[dir][c] + g[c][dir]);
    const FT en = fma(uh[0], sg[0], fma(uh[1], sg[1], fma(uh[2], sg[2], arg_ft<FT>(D.kappa, D.kappa_f) * Tn)));
    Fn[1] = Fn[1] - sg[dir];
    Fn[2] = Fn[2] - sg[t1];
    Fn[3] = Fn[3] - sg[t2];
    Fn[4] = Fn[4] - en;
}

// Face frame -> (rho, rho u, rho v, rho w, rho E).
template <class FT, int dir>
__device__ __forceinline__ void from_frame(const FT Fn[NV3], FT F[NV3])
{
    constexpr int t1 = (dir + 1) % 3, t2 = (dir + 2) % 3;
    F[0] = Fn[0];
    F[1 + dir] = Fn[1];
    F[1 + t1] = Fn[2];
    F[1 + t2] = Fn[3];
    F[4] = Fn[4];
}

// x- (dir 0) or y-face (dir 1) between staged-plane cell (x, y) and its +dir
// neighbour.  Q: the plane's state slot [5][HY][HX]; Pm, P0, Pp: primitive
// slots [4][PY][PX] of planes z-1, z, z+1.
template <class FT, int dir, class S>
__device__ __forceinline__ void face_xy(const StageArgs& A, const DomainArgs& D, const FT* Q, const FT* Pm,
                                        const FT* P0, const FT* Pp, int x, int y, FT F[NV3])
{
#pragma clang fp contract(off)
    constexpr int t1 = (dir + 1) % 3, t2 = (dir + 2) % 3;
    constexpr int comp[NV3] = {0, 1 + dir, 1 + t1, 1 + t2, 4};
    constexpr int sn = dir == 0 ? 1 : S::HX;
    const FT q4 = FT(0.25), h = FT(0.5);
    FT qL[NV3], qR[NV3];
    const int qb = (y + 2) * S::HX + x + 2;
#pragma unroll
    for (int k = 0; k < NV3; ++k) {
        const FT* s = Q + comp[k] * S::QPL + qb;
        const FT qm = s[-sn], q0 = s[0], q1 = s[sn], q2 = s[2 * sn];
        qL[k] = fma(q4, q1 - qm, q0);
        qR[k] = fma(-q4, q2 - q0, q1);
    }
    FT Fn[NV3];
    llf3n<FT>(A, qL, qR, F3_INTERIOR, Fn);
    // Keep the gradient loads after the inviscid part (register pressure).
    __builtin_amdgcn_sched_barrier(0);
    constexpr int pn = dir == 0 ? 1 : S::PX;      // normal stride in a primitive plane
    constexpr int pt = dir == 0 ? S::PX : 1;      // in-plane tangential stride
    const int pb = (y + 1) * S::PX + x + 1;
    const FT inv_h[3] = {arg_ft<FT>(A.inv_dx, A.inv_dx_f), arg_ft<FT>(A.inv_dy, A.inv_dy_f),
                         arg_ft<FT>(D.inv_dz, D.inv_dz_f)};
    FT g[3][3], uh[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const FT* U = P0 + c * S::PPL + pb;
        const FT* Um = Pm + c * S::PPL + pb;
        const FT* Up = Pp + c * S::PPL + pb;
        uh[c] = h * (U[0] + U[pn]);
        g[c][dir] = (U[pn] - U[0]) * inv_h[dir];
        g[c][1 - dir] = ((U[pt] - U[-pt]) + (U[pn + pt] - U[pn - pt])) * (q4 * inv_h[1 - dir]);
        g[c][2] = ((Up[0] - Um[0]) + (Up[pn] - Um[pn])) * (q4 * inv_h[2]);
    }
    const FT* Tt = P0 + 3 * S::PPL + pb;
    const FT Tn = (Tt[pn] - Tt[0]) * inv_h[dir];
    visc3n<FT, dir>(D, uh, g, Tn, Fn);
    from_frame<FT, dir>(Fn, F);
}

// z-face above column cell (x, y) of plane z: the column's states at planes
// z-1, z, z+1, z+2 (c0..c3, components rho, rho u, rho v, rho w, rho E) and
// the primitive slots of planes z (Pa) and z+1 (Pb).
template <class FT, class S>
__device__ __forceinline__ void face_z(const StageArgs& A, const DomainArgs& D, const FT* c0, const FT* c1,
                                       const FT* c2, const FT* c3, const FT* Pa, const FT* Pb, int x, int y,
                                       int kind, FT F[NV3])
{
#pragma clang fp contract(off)
    constexpr int comp[NV3] = {0, 3, 1, 2, 4};
    const FT q4 = FT(0.25), h = FT(0.5);
    FT qL[NV3], qR[NV3];
#pragma unroll
    for (int k = 0; k < NV3; ++k) {
        const int v = comp[k];
        qL[k] = fma(q4, c2[v] - c0[v], c1[v]);
        qR[k] = fma(-q4, c3[v] - c1[v], c2[v]);
    }
    FT Fn[NV3];
    llf3n<FT>(A, qL, qR, kind, Fn);
    __builtin_amdgcn_sched_barrier(0);
    if (kind == F3_INTERIOR) {
        FT g[3][3], uh[3];
        const int pb = (y + 1) * S::PX + x + 1;
        const FT inv_h[3] = {arg_ft<FT>(A.inv_dx, A.inv_dx_f), arg_ft<FT>(A.inv_dy, A.inv_dy_f),
                             arg_ft<FT>(D.inv_dz, D.inv_dz_f)};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const FT* U = Pa + c * S::PPL + pb;
            const FT* V = Pb + c * S::PPL + pb;
            uh[c] = h * (U[0] + V[0]);
            g[c][2] = (V[0] - U[0]) * inv_h[2];
            g[c][0] = ((U[1] - U[-1]) + (V[1] - V[-1])) * (q4 * inv_h[0]);
            g[c][1] = ((U[S::PX] - U[-S::PX]) + (V[S::PX] - V[-S::PX])) * (q4 * inv_h[1]);
        }
        const FT Tn = (Pb[3 * S::PPL + pb] - Pa[3 * S::PPL + pb]) * inv_h[2];
        visc3n<FT, 2>(D, uh, g, Tn, Fn);
    }
    from_frame<FT, 2>(Fn, F);
}

// Stage results of the marching kernel: as st_dev, but the ordinary store is
// non-temporal, and the substep base is read non-temporally too, so that the
// staged planes, which neighbouring tiles read again, keep more of the L2
// (1.5% per slow step on the 256 x 256 x 128 x 2 workload).
__device__ __forceinline__ void st_march(bool dev, double* p, double x)
{
    if (dev) __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else __builtin_nontemporal_store(x, p);
}

template <int DOM, class FT, class S>
__device__ __forceinline__ void march_tile3(const StageArgs& A, int tile, char* smem)
{
    constexpr int TX = S::TX, TY = S::TY, LZ = S::LZ, NT = S::NT;
    constexpr int HX = S::HX, QPL = S::QPL, PX = S::PX, PPL = S::PPL, NPOS = S::NPOS;
    const DomainArgs& D = A.d[DOM];
    const DomainArgs& O = A.d[1 - DOM];
    const int tid = threadIdx.x;
    const int nx = A.nx, ny = A.ny, nz = D.nz;
    // Block -> (segment, x-y tile): the x-y tiles of one segment layer are
    // consecutive (x fastest), so the workgroups that one XCD runs at a time
    // are x-y neighbours and share their halo columns in its L2.
    const int nxy = D.tiles_x * D.tiles_y;
    const int seg = tile / nxy;
    const int txy = tile - seg * nxy;
    const int ty = txy / D.tiles_x, tx = txy - ty * D.tiles_x;
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = (D.row_lo / LZ + seg) * LZ;
    const int zs = max(z0, D.row_lo), ze = min(z0 + LZ, D.row_hi);
    const int ncx = min(TX, nx - x0), ncy = min(TY, ny - y0);
    const size_t rowsz = (size_t)ny * nx;

    FT* Lq = (FT*)smem;                       // [2][5][HY][HX]
    FT* Lp = Lq + S::LDS_Q;                   // [3][4][PY][PX]
    FT* ex_x = Lp + S::LDS_P;                 // [5][TY][TX+1]
    FT* ex_y = ex_x + NV3 * S::EXX;           // [5][TY+1][TX]
    double* gf = (double*)(smem + (S::LDS_Q + S::LDS_P + S::LDS_X) * sizeof(FT));   // [3][TY*TX]

    const int cx = tid % TX, cy = tid / TX;
    const bool own = cx < ncx && cy < ncy;
    const bool near = nx > TX && ny > TY;

    // Staged positions of this thread (fixed for the segment): first its own
    // cell, then, for the first QPL - NT threads, one cell of the 2-cell ring
    // around the tile (the two rows below it, the two rows above it, then the
    // two cells left and right of each row).
    static_assert(NPOS == 2 && QPL - NT <= NT, "one own cell and at most one ring cell per thread");
    constexpr int NRING = QPL - NT;
    uint32_t cofs[NPOS];   // offset in a plane (a domain holds at most 2^28 cells)
    int qpos[NPOS];   // index in a staged plane
    int ppos[NPOS];   // primitive index in a plane, or -1 outside the 1-cell ring
#pragma unroll
    for (int k = 0; k < NPOS; ++k) {
        int xx, yy;
        if (k == 0) {
            xx = cx + 2;
            yy = cy + 2;
        } else if (tid < 2 * HX) {
            yy = tid / HX;
            xx = tid - yy * HX;
        } else if (tid < 4 * HX) {
            const int r = tid - 2 * HX;
            yy = S::HY - 2 + r / HX;
            xx = r - (r / HX) * HX;
        } else {
            const int s = min(tid, NRING - 1) - 4 * HX, j = s & 3;
            yy = 2 + (s >> 2);
            xx = j < 2 ? j : HX - 4 + j;
        }
        const int col = near ? wrap1(x0 + xx - 2, nx) : wrapx(x0 + xx - 2, nx);
        const int rowy = near ? wrap1(y0 + yy - 2, ny) : wrapx(y0 + yy - 2, ny);
        cofs[k] = (uint32_t)(rowy * nx + col);
        qpos[k] = yy * HX + xx;
        ppos[k] = (xx >= 1 && xx <= HX - 2 && yy >= 1 && yy <= S::HY - 2) ? (yy - 1) * PX + xx - 1 : -1;
    }
    const bool ring = tid < NRING;

    // Global loads of plane p (mirror planes beyond the domain, retained slow
    // planes at substeps 2..m) into registers; returns the mirror flag.
    auto load_plane = [&](int p, double (&val)[NPOS][NV3]) -> bool {
        int pl = p;
        bool neg = false;
        if (pl < 0) { pl = 0; neg = true; }
        else if (pl >= nz) { pl = nz - 1; neg = true; }
        const double* src;
        size_t vstride;
        if (D.use_ret && (pl < D.b_lo || pl >= D.b_hi)) {
            int rr = pl - D.ret_lo;
            rr = rr < 0 ? 0 : (rr > 1 ? 1 : rr);
            src = D.ret_in + (size_t)rr * rowsz;
            vstride = 2 * rowsz;
        } else {
            src = D.qin + (size_t)pl * rowsz;
            vstride = (size_t)nz * rowsz;
        }
#pragma unroll
        for (int k = 0; k < NPOS; ++k)
            if (k == 0 || ring) {
#pragma unroll
                for (int v = 0; v < NV3; ++v) val[k][v] = src[(size_t)cofs[k] + v * vstride];
            }
        return neg;
    };
    // Plane p into its state slot (p & 1) and, from the same values, its
    // primitives into primitive slot (p + 3) % 3; mine receives the own
    // cell's staged values and lo the low words of their FP64 values (FP32
    // staging).
    auto commit_plane = [&](int p, const double (&val)[NPOS][NV3], bool neg, FT (&mine)[NV3],
                            uint32_t (&lo)[NV3]) {
        FT* Q = Lq + (p & 1) * NV3 * QPL;
        FT* P = Lp + ((p + 3) % 3) * 4 * PPL;
#pragma unroll
        for (int k = 0; k < NPOS; ++k) {
            if (k == 0 || ring) {
                FT c[NV3];
#pragma unroll
                for (int v = 0; v < NV3; ++v) {
                    const double x = (v == 3 && neg) ? -val[k][v] : val[k][v];
                    c[v] = FT(x);
                    Q[v * QPL + qpos[k]] = c[v];
                    if (k == 0) mine[v] = c[v];
                    if constexpr (sizeof(FT) == 4) {
                        if (k == 0) lo[v] = low_word(x, c[v]);
                    }
                }
                if (ppos[k] >= 0) {
                    FT pu, pv, pw, pT;
                    prim3<FT>(c, arg_ft<FT>(A.gamma, A.gamma_f), arg_ft<FT>(A.gm1, A.gm1_f), pu, pv, pw,
                              pT);
                    P[ppos[k]] = pu;
                    P[PPL + ppos[k]] = pv;
                    P[2 * PPL + ppos[k]] = pw;
                    P[3 * PPL + ppos[k]] = pT;
                }
            }
        }
    };
    const int qown = (cy + 2) * HX + cx + 2;
    auto read_col = [&](int p, FT (&c)[NV3]) {
        const FT* Q = Lq + (p & 1) * NV3 * QPL;
#pragma unroll
        for (int v = 0; v < NV3; ++v) c[v] = Q[v * QPL + qown];
    };
    auto pslot = [&](int p) -> const FT* { return Lp + ((p + 3) % 3) * 4 * PPL; };

    __builtin_amdgcn_s_setprio(2);
    // Interface flux per column (FP64 from the FP64 cells next to the lid),
    // when the segment holds the row next to it.
    const bool has_gamma = (DOM == 0) ? (D.gamma_top && ze == nz) : (D.gamma_bot && zs == 0);
    if (has_gamma && tid < TX * TY) {
        const int xx = tid % TX, yy = tid / TX;
        const int col = near ? wrap1(x0 + xx, nx) : wrapx(x0 + xx, nx);
        const int rowy = near ? wrap1(y0 + yy, ny) : wrapx(y0 + yy, ny);
        const int ownp = (DOM == 0) ? nz - 1 : 0;
        const int oth = (DOM == 0) ? 0 : O.nz - 1;
        const size_t po = (size_t)nz * rowsz, pq = (size_t)O.nz * rowsz;
        const double* a = D.qin + (size_t)ownp * rowsz + (size_t)rowy * nx + col;
        const double* b = O.qin + (size_t)oth * rowsz + (size_t)rowy * nx + col;
        double ca[NV3], cb[NV3];
#pragma unroll
        for (int v = 0; v < NV3; ++v) { ca[v] = a[v * po]; cb[v] = b[v * pq]; }
        double ua, va, Ta, ub, vb, Tb, f[3];
        interface_cell3(ca, A.gamma, A.gm1, ua, va, Ta);
        interface_cell3(cb, A.gamma, A.gm1, ub, vb, Tb);
        if (DOM == 0) interface_flux3(A, ua, va, Ta, ub, vb, Tb, f);
        else interface_flux3(A, ub, vb, Tb, ua, va, Ta, f);
        gf[tid] = f[0];
        gf[TX * TY + tid] = f[1];
        gf[2 * TX * TY + tid] = f[2];
    }

    // ---- prologue: planes zs-2 .. zs+1, and the z-face below zs.  The own
    // column comes from the thread's own staged cells; plane zs+1 overwrites
    // the primitives of plane zs-2, which no face of this segment reads.
    FT cm[NV3], c0[NV3], c1[NV3], c2[NV3];   // column: planes z-1, z (kept), z+1 (from LDS), z+2 (own commit)
    uint32_t lo0[NV3], lo1[NV3], lo2[NV3];    // low words of the own cell at planes z, z+1, z+2
    double va[NPOS][NV3];
    {
        FT cmm[NV3];
        // (planes zs-2 and zs-1 are never combined here: their low words go to
        // lo0, which plane zs then overwrites)
        bool na = load_plane(zs - 2, va);
        commit_plane(zs - 2, va, na, cmm, lo0);
        na = load_plane(zs - 1, va);
        commit_plane(zs - 1, va, na, cm, lo0);
        na = load_plane(zs, va);
        commit_plane(zs, va, na, c0, lo0);
        na = load_plane(zs + 1, va);
        commit_plane(zs + 1, va, na, c1, lo1);
        __syncthreads();
        // the z-face below the first plane (bottom wall or lid when zs == 0)
        FT Fb[NV3];
        face_z<FT, S>(A, D, cmm, cm, c0, c1, pslot(zs - 1), pslot(zs), cx, cy,
                      zs == 0 ? F3_BOTTOM : F3_INTERIOR, Fb);
#pragma unroll
        for (int v = 0; v < NV3; ++v) c2[v] = Fb[v];   // c2 holds the lower face until the loop
    }
    FT Fbot[NV3];
#pragma unroll
    for (int v = 0; v < NV3; ++v) Fbot[v] = c2[v];
    __builtin_amdgcn_s_setprio(0);

    const double inv_dx = A.inv_dx, inv_dy = A.inv_dy, inv_dz = D.inv_dz;
    const int col = x0 + cx, rowy = y0 + cy;
    const size_t plane = (size_t)nz * rowsz;
    const size_t nbx = (size_t)(D.b_hi - D.b_lo) * rowsz;

    for (int z = zs; z < ze; ++z) {
        // Global loads of plane z+2 (staged after this plane's x-y faces).
        __builtin_amdgcn_s_setprio(2);
        const bool nload = load_plane(z + 2, va);
        __builtin_amdgcn_s_setprio(0);

        // ---- x and y faces of plane z (own +x, +y; edge faces x = -1 in
        // wave 0, y = -1 in wave 1), each written to the exchange at once (the
        // previous plane's exchange reads ended at the last barrier).
        {
            const FT* Q = Lq + (z & 1) * NV3 * QPL;
            const FT* Pm = pslot(z - 1);
            const FT* P0 = pslot(z);
            const FT* Pp = pslot(z + 1);
            FT F[NV3];
            if (own) {
                face_xy<FT, 0, S>(A, D, Q, Pm, P0, Pp, cx, cy, F);
                FT* e = ex_x + cy * (TX + 1) + cx + 1;
#pragma unroll
                for (int v = 0; v < NV3; ++v) e[v * S::EXX] = F[v];
                face_xy<FT, 1, S>(A, D, Q, Pm, P0, Pp, cx, cy, F);
                FT* f = ex_y + (cy + 1) * TX + cx;
#pragma unroll
                for (int v = 0; v < NV3; ++v) f[v * S::EXY] = F[v];
            }
            if (tid < ncy) {
                face_xy<FT, 0, S>(A, D, Q, Pm, P0, Pp, -1, tid, F);
                FT* e = ex_x + tid * (TX + 1);
#pragma unroll
                for (int v = 0; v < NV3; ++v) e[v * S::EXX] = F[v];
            }
            if (tid >= 64 && tid - 64 < ncx) {
                face_xy<FT, 1, S>(A, D, Q, Pm, P0, Pp, tid - 64, -1, F);
                FT* f = ex_y + (tid - 64);
#pragma unroll
                for (int v = 0; v < NV3; ++v) f[v * S::EXY] = F[v];
            }
            __syncthreads();   // plane z's state slot and plane z-1's primitives are free
        }
        // Plane z+2 into the freed slots.  What follows reads neither of them
        // (the z-face takes plane z+2 from this thread's own commit), so the
        // next barrier, at the end of the plane, also publishes this commit.
        commit_plane(z + 2, va, nload, c2, lo2);

        // The FP64 stage value of plane z (rebuilt from its FP32 copy and low
        // word; read from memory where that declines) and the substep base U.
        const bool inb = (z >= D.b_lo && z < D.b_hi);
        const Combine cb = pick_combine(D.buf, D.main, inb);
        const size_t id = (size_t)z * rowsz + (size_t)rowy * nx + col;
        double qc[NV3], Ub[NV3];
#pragma unroll
        for (int v = 0; v < NV3; ++v) Ub[v] = 0.0;
        if constexpr (sizeof(FT) == 4) {
            bool ok[NV3], all = true;
#pragma unroll
            for (int v = 0; v < NV3; ++v) {
                qc[v] = join_low(c0[v], lo0[v], ok[v]);
                all = all && ok[v];
            }
            if (own && !all) {
#pragma unroll
                for (int v = 0; v < NV3; ++v)
                    if (!ok[v]) qc[v] = D.qin[v * plane + id];
            }
        } else {
#pragma unroll
            for (int v = 0; v < NV3; ++v) qc[v] = (double)c0[v];
        }
        if (own && cb.mode != MODE_RHS && cb.alpha != 0.0) {
#pragma unroll
            for (int v = 0; v < NV3; ++v) Ub[v] = __builtin_nontemporal_load(&D.base[v * plane + id]);
        }

        // ---- z-face above plane z, divergence, source, combination.
        read_col(z + 1, c1);   // slot (z + 1) & 1, committed at the previous plane
        FT Ftop[NV3];
        face_z<FT, S>(A, D, cm, c0, c1, c2, pslot(z), pslot(z + 1), cx, cy,
                      z == nz - 1 ? F3_TOP : F3_INTERIOR, Ftop);
        if (own) {
            double R[NV3];
#pragma unroll
            for (int v = 0; v < NV3; ++v) {
                const FT* fx = ex_x + v * S::EXX + cy * (TX + 1) + cx;
                const FT* fy = ex_y + v * S::EXY + cy * TX + cx;
                R[v] = -((double)fx[1] - (double)fx[0]) * inv_dx -
                       ((double)fy[TX] - (double)fy[0]) * inv_dy -
                       ((double)Ftop[v] - (double)Fbot[v]) * inv_dz;
            }
            const int gc = cy * TX + cx;
            if (DOM == 0 && D.gamma_top && z == nz - 1) {
                R[1] += gf[gc] * inv_dz;
                R[2] += gf[TX * TY + gc] * inv_dz;
                R[4] += gf[2 * TX * TY + gc] * inv_dz;
            }
            if (DOM == 1 && D.gamma_bot && z == 0) {
                R[1] -= gf[gc] * inv_dz;
                R[2] -= gf[TX * TY + gc] * inv_dz;
                R[4] -= gf[2 * TX * TY + gc] * inv_dz;
            }
            R[3] += qc[0] * A.gravity;
            R[4] += qc[3] * A.gravity;
            if (cb.mode == MODE_RHS) {
#pragma unroll
                for (int v = 0; v < NV3; ++v) st_march(A.dev_stores != 0, &D.out[v * plane + id], R[v]);
            } else if (cb.alpha == 0.0) {
#pragma unroll
                for (int v = 0; v < NV3; ++v)
                    st_march(A.dev_stores != 0, &D.out[v * plane + id], qc[v] + cb.bh * R[v]);
            } else {
                double inc[NV3];
#pragma unroll
                for (int v = 0; v < NV3; ++v) inc[v] = cb.beta * (qc[v] - Ub[v]) + cb.bh * R[v];
                if (cb.mode == MODE_STAGE) {
#pragma unroll
                    for (int v = 0; v < NV3; ++v) st_march(A.dev_stores != 0, &D.out[v * plane + id], Ub[v] + inc[v]);
                } else {
                    const size_t ia = (size_t)(z - D.b_lo) * rowsz + (size_t)rowy * nx + col;
                    if (cb.mode == MODE_ACC_FIRST) {
#pragma unroll
                        for (int v = 0; v < NV3; ++v) st_march(A.dev_stores != 0, &D.acc[v * nbx + ia], inc[v]);
                    } else if (cb.mode == MODE_ACC_ADD) {
#pragma unroll
                        for (int v = 0; v < NV3; ++v)
                            st_march(A.dev_stores != 0, &D.acc[v * nbx + ia], D.acc[v * nbx + ia] + inc[v]);
                    } else {
#pragma unroll
                        for (int v = 0; v < NV3; ++v)
                            st_march(A.dev_stores != 0, &D.out[v * plane + id],
                                   Ub[v] + (D.acc[v * nbx + ia] + inc[v]) * A.inv_m);
                    }
                }
            }
            if (D.ret_out && z >= D.ret_lo && z < D.ret_lo + 2) {
#pragma unroll
                for (int v = 0; v < NV3; ++v)
                    st_march(A.dev_stores != 0,
                           &D.ret_out[(size_t)(v * 2 + z - D.ret_lo) * rowsz + (size_t)rowy * nx + col], qc[v]);
            }
        }
#pragma unroll
        for (int v = 0; v < NV3; ++v) {
            Fbot[v] = Ftop[v];
            cm[v] = c0[v];
            c0[v] = c1[v];
            lo0[v] = lo1[v];
            lo1[v] = lo2[v];
        }
        __syncthreads();   // exchange reads done and plane z+2 published before the next plane's faces
    }
}

template <class FT, class S>
__global__ __launch_bounds__(S::NT) __attribute__((amdgpu_waves_per_eu(MPRK3_MARCH_WAVES))) void march_kernel3(const StageArgs A)
{
    __shared__ __align__(16) char smem[S::template lds_bytes<FT>()];
    const int b = xcd_contiguous(blockIdx.x, A.nblocks);
    const int n0 = A.d[A.first].ntiles;
    const int dom = (b < n0) ? A.first : 1 - A.first;
    const int t = (b < n0) ? b : b - n0;
    if (dom == 0) march_tile3<0, FT, S>(A, t, smem);
    else march_tile3<1, FT, S>(A, t, smem);
}

}  // namespace

hipError_t launch_stage3(const StageArgs& a, hipStream_t s)
{
    if (a.nblocks <= 0) return hipSuccess;
    if (a.flux32) hipLaunchKernelGGL((march_kernel3<float, M32>), dim3(a.nblocks), dim3(M32::NT), 0, s, a);
    else hipLaunchKernelGGL(stage_kernel3<double>, dim3(a.nblocks), dim3(T64::NT), 0, s, a);
    return hipGetLastError();
}

KernelRef stage3_kernel_ref(bool flux32)
{
    if (flux32) return KernelRef{(const void*)march_kernel3<float, M32>, M32::NT};
    return KernelRef{(const void*)stage_kernel3<double>, T64::NT};
}

TileDims3 tile3_dims(bool flux32)
{
    if (flux32) return {M32::TX, M32::TY, M32::LZ, M32::NT};
    return {T64::TX, T64::TY, T64::TZ, T64::NT};
}

}  // namespace mprk
