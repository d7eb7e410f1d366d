// mprk_kernels.hip -- gfx950 kernels of the MPRK library.
//
// stage_kernel: one MPRK stage for every cell a launch covers, in both
// domains at once.  For each cell: the coupled finite-volume RHS (Section 2.1,
// Appendix B restricted to x-z; local Lax-Friedrichs flux with Roe-average
// wave speed, common-value viscous flux, bulk-coefficient interface flux of
// eq. bulk-flux) and the stage combination of its partition (eq. MRK2 in a
// low-storage substep form).
//
// Tiling: a workgroup of 512 threads owns a 32 x 16 tile of one domain, one
// cell per thread (other tile shapes and cells-per-thread counts are template
// parameters).  The tile's conserved state (2-cell halo) is staged in LDS,
// and the loader threads compute the primitives u, w, T of the tile and its
// 1-cell ring from the values they stage (no separate pass); every face of
// the tile is computed exactly once (two faces per cell plus one left column
// and one bottom row of edge faces) by a single direction-generic face
// routine; the fluxes are exchanged through LDS (aliasing the staged state)
// and each thread forms the divergence of its cells from its own two face
// fluxes (registers) and its neighbours' two (LDS).  Three barriers per
// tile.  One cell per thread keeps the register count low (74 VGPRs in FP64,
// 50 in FP32), so more waves hide the LDS and HBM latency than with two
// cells per thread.
//
// reduce_*: deterministic (fixed-order) device reductions for the totals,
// stability measures and the physical-state flag.
#include <mutex>

#include "mprk_internal.h"
#include "mprk_device.h"

namespace mprk {

namespace {

template <int X, int Z, int C = 1>
struct Shape {
    static constexpr int CZ = C;                      // cells per thread, stacked in z
    static constexpr int TX = X, TZ = Z, NT = X * Z / C;
    static constexpr int HX = X + 4, HZ = Z + 4;      // staged state with a 2-cell halo
    static constexpr int PX = X + 2, PZ = Z + 2;      // primitives with a 1-cell halo
    static constexpr int LDS_Q = NV * HZ * HX;        // staged conserved state
    static constexpr int LDS_P = 3 * PZ * PX;         // staged primitives u, w, T
    static constexpr int LDS_EX = NV * Z * (X + 1) + NV * (Z + 1) * X;  // face fluxes
    static_assert(Z % C == 0 && NT % 64 == 0 && NT <= 1024, "tile shape");
    static_assert(NT >= X + Z, "one edge face per thread of the first X + Z");
    static_assert(LDS_EX <= LDS_Q + LDS_P, "flux exchange must fit in the staged state");
    // Shared memory of one tile: the staged state and primitives in the flux
    // type FT (the flux exchange reuses that space), then the per-column
    // interface flux in FP64.
    template <class FT>
    static constexpr int lds_bytes() { return (LDS_Q + LDS_P) * (int)sizeof(FT) + 2 * X * 8; }
};

// Brings a shape's constants into a function's scope.
#define MPRK_SHAPE_CONSTANTS(S)                                                          \
    constexpr int TX = S::TX, TZ = S::TZ, NT = S::NT, HX = S::HX, HZ = S::HZ;            \
    constexpr int PX = S::PX, PZ = S::PZ;                                                \
    (void)TX; (void)TZ; (void)NT; (void)HX; (void)HZ; (void)PX; (void)PZ

// Cell primitives u, w, T in the flux type (staged for the viscous fluxes).
// A cell's primitives are computed by every tile that stages it; contraction
// is off and the fused operations are written out, so every tile obtains the
// same bits (the face fluxes built from them must agree across tiles).
template <class FT>
__device__ __forceinline__ void primitives(FT rho, FT mx, FT mz, FT en, FT gamma, FT gm1, FT& u,
                                           FT& w, FT& T)
{
#pragma clang fp contract(off)
    const FT ir = Fm<FT>::rcp(rho);
    u = mx * ir;
    w = mz * ir;
    const FT p = gm1 * fma(FT(-0.5), fma(mx, u, mz * w), en);
    T = gamma * p * ir;
}

// FP64 u and T of a cell next to the interface.  Contraction is off and the
// same code runs in the tiles on both sides, so both obtain the same bits.
__device__ __forceinline__ void interface_cell(double rho, double mx, double mz, double en,
                                               double gamma, double gm1, double& u, double& T)
{
#pragma clang fp contract(off)
    const double ir = rcp_nr(rho);
    u = mx * ir;
    const double w = mz * ir;
    const double p = gm1 * (en - 0.5 * (mx * u + mz * w));
    T = gamma * p * ir;
}

// Interface viscous flux in +z (Appendix B, eq. bulk-flux; hat w = 0 and
// hat sigma_zz = 0 on the lid): (0, sigma_xz, 0, u_w sigma_xz - Pi_z) with
// sigma_xz = b_u (u2 - u1), Pi_z = -b_T (T2 - T1), u_w = u1 + sigma dz1/(2 mu1).
// Index 1 is the lower cell, 2 the upper cell.  FP64, contraction off: both
// domains evaluate it and must obtain the same bits (exact exchange).
__device__ __forceinline__ void interface_flux(const StageArgs& A, double u1, double T1,
                                               double u2, double T2, double& f1, double& f3)
{
#pragma clang fp contract(off)
    double sig = A.bu * (u2 - u1);
    double pi = -A.bT * (T2 - T1);
    double uw = u1 + sig * A.half_dz1_mu1;
    f1 = sig;
    f3 = uw * sig - pi;
}

template <class FT>
struct Lds {
    FT* q;        // [NV][HZ][HX]
    FT* p;        // [3][PZ][PX]
    double* gf;   // [2][TX]: interface flux (x-momentum, energy) per column
};

template <class S>
__device__ __forceinline__ int qidx(int v, int r, int c) { return (v * S::HZ + r + 2) * S::HX + c + 2; }
template <class S>
__device__ __forceinline__ int pidx(int f, int r, int c) { return (f * S::PZ + r + 1) * S::PX + c + 1; }

// Boundary kinds of a face.
enum : int { FACE_INTERIOR = 0, FACE_TOP = 1, FACE_BOTTOM = 2 };

// Twice the numerical flux (inviscid minus viscous) through the face between
// tile cell (c, r) and its +dir neighbour (dir 0: x, 1: z; a constant at the
// interior call sites, a per-lane value for the edge faces), in the
// face-normal frame: returns 2 (F_rho, F_normal-momentum,
// F_tangential-momentum, F_energy), in FT.  The factor 2 is exact in binary
// floating point and saves the halvings of the central averages; the
// divergence takes it back with the half inverse spacings.
//   kind FACE_TOP:    (c, r) is the top interior row; the other side is its
//                     mirror (wall or interface).
//   kind FACE_BOTTOM: (c, r+1) is the bottom interior row; likewise.
// At walls and at the interface the viscous part is not added here: walls
// carry none, and the interface flux enters the divergence in FP64.
template <class FT, class S>
__device__ __forceinline__ void face_flux(const StageArgs& A, const DomainArgs& D, const Lds<FT>& L,
                                          int dir, int c, int r, int kind, FT F[NV])
{
    // A face on a tile edge is computed by the tiles on both sides, at
    // different call sites.  With contraction off and the fused operations
    // written out, every call site performs the same IEEE operations, so both
    // obtain the same bits and the flux differences telescope exactly.
#pragma clang fp contract(off)
    MPRK_SHAPE_CONSTANTS(S);
    const FT gamma = arg_ft<FT>(A.gamma, A.gamma_f), gm1 = arg_ft<FT>(A.gm1, A.gm1_f);
    const FT h = FT(0.5), q4 = FT(0.25);
    const int sn = dir ? HX : 1;             // normal stride in the state tile
    const int vn = dir ? 2 : 1;              // normal momentum component
    const int vt = dir ? 1 : 2;              // tangential momentum component
    constexpr int plane = HZ * HX;
    const int comp[NV] = {0, vn, vt, 3};

    // Reconstruction of conserved variables with central cell gradients:
    // qL = q_c + (q_{c+1} - q_{c-1})/4, qR = q_{c+1} - (q_{c+2} - q_c)/4.
    FT qL[NV], qR[NV];
    const int base = qidx<S>(0, r, c);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const FT* s = L.q + comp[k] * plane + base;
        const FT qm = s[-sn], q0 = s[0], q1 = s[sn], q2 = s[2 * sn];
        qL[k] = fma(q4, q1 - qm, q0);
        qR[k] = fma(-q4, q2 - q0, q1);
    }
    if (kind == FACE_TOP) {
        qR[0] = qL[0]; qR[1] = -qL[1]; qR[2] = qL[2]; qR[3] = qL[3];
    } else if (kind == FACE_BOTTOM) {
        qL[0] = qR[0]; qL[1] = -qR[1]; qL[2] = qR[2]; qL[3] = qR[3];
    }

    // Local Lax-Friedrichs flux, lambda = max(|u_n| + a) over qL, qR and the
    // Roe average (sqrt(rho)-weighted velocity and total enthalpy; the
    // weighted numerators are sqrt(rho) phi = (rho phi) / sqrt(rho)).  One
    // reciprocal square root per side gives 1/rho, 1/sqrt(rho), sqrt(rho).
    FT rL, yL, sL, rR, yR, sR;
    Fm<FT>::inv_sqrt(qL[0], rL, yL, sL);
    Fm<FT>::inv_sqrt(qR[0], rR, yR, sR);
    const FT unL = qL[1] * rL, utL = qL[2] * rL;
    const FT unR = qR[1] * rR, utR = qR[2] * rR;
    const FT pL = gm1 * fma(-h, fma(qL[1], unL, qL[2] * utL), qL[3]);
    const FT pR = gm1 * fma(-h, fma(qR[1], unR, qR[2] * utR), qR[3]);
    const FT eL = qL[3] + pL, eR = qR[3] + pR;   // rho H
    const FT aL = Fm<FT>::ws_sqrt(gamma * pL * rL);
    const FT aR = Fm<FT>::ws_sqrt(gamma * pR * rR);
    const FT iw = Fm<FT>::ws_rcp(sL + sR);
    const FT unr = fma(qL[1], yL, qR[1] * yR) * iw;
    const FT utr = fma(qL[2], yL, qR[2] * yR) * iw;
    const FT Hr = fma(eL, yL, eR * yR) * iw;
    const FT ar = Fm<FT>::ws_sqrt(gm1 * fma(-h, fma(unr, unr, utr * utr), Hr));
    const FT lam = fmax(fmax(fabs(unL) + aL, fabs(unR) + aR), fabs(unr) + ar);
    if (kind != FACE_INTERIOR) {
        // Against its mirror image the flux reduces exactly to
        // (0, rho u_n^2 + p +- lambda rho u_n, 0, 0); the closed form keeps
        // the mass, tangential-momentum and energy fluxes at exactly zero,
        // where the general formula leaves rounding residuals.
        F[0] = FT(0);
        F[1] = FT(2) * ((kind == FACE_TOP) ? fma(lam, qL[1], fma(qL[1], unL, pL))
                                           : fma(-lam, qR[1], fma(qR[1], unR, pR)));
        F[2] = FT(0);
        F[3] = FT(0);
        return;
    }
    F[0] = fma(-lam, qR[0] - qL[0], qL[1] + qR[1]);
    F[1] = fma(-lam, qR[1] - qL[1], fma(qL[1], unL, qR[1] * unR) + (pL + pR));
    F[2] = fma(-lam, qR[2] - qL[2], fma(qL[2], unL, qR[2] * unR));
    F[3] = fma(-lam, qR[3] - qL[3], fma(eL, unL, eR * unR));

    {
        // Common values: averaged velocity, normal derivative by finite
        // difference, tangential derivative by averaging cell gradients; the
        // spacings and mu, kappa are folded into the coefficients vk.
        const int pb = pidx<S>(0, r, c);
        const int pn = dir ? PX : 1;
        const int pt = dir ? 1 : PX;
        const int fn = dir ? 1 : 0;          // normal velocity in the primitive tile
        const int ft = dir ? 0 : 1;
        // Coefficient of the normal (n) or tangential (t) direction: both are
        // read as uniform arguments and selected per lane (edge faces).
        auto vkn = [&](int row) { const FT x = arg_vk<FT>(D, row, 0), z = arg_vk<FT>(D, row, 2); return dir ? z : x; };
        auto vkt = [&](int row) { const FT x = arg_vk<FT>(D, row, 0), z = arg_vk<FT>(D, row, 2); return dir ? x : z; };
        constexpr int pp = PZ * PX;
        const FT* Un = L.p + fn * pp + pb;
        const FT* Ut = L.p + ft * pp + pb;
        const FT* Tt = L.p + 2 * pp + pb;
        const FT unA = Un[0], unB = Un[pn], utA = Ut[0], utB = Ut[pn];
        const FT t_un = (Un[pt] - Un[-pt]) + (Un[pn + pt] - Un[pn - pt]);
        const FT t_ut = (Ut[pt] - Ut[-pt]) + (Ut[pn + pt] - Ut[pn - pt]);
        const FT snn = fma(vkn(VK_NN), unB - unA, vkt(VK_TT) * t_ut);
        const FT snt = fma(vkn(VK_N), utB - utA, vkt(VK_TN) * t_un);
        F[1] = fma(FT(-2), snn, F[1]);
        F[2] = fma(FT(-2), snt, F[2]);
        F[3] = F[3] - fma(unA + unB, snn, fma(utA + utB, snt, vkn(VK_Q) * (Tt[pn] - Tt[0])));
    }
}

template <int DOM, class FT, class S>
__device__ __forceinline__ void stage_tile(const StageArgs& A, int tile, char* smem)
{
    MPRK_SHAPE_CONSTANTS(S);
    constexpr int LDS_Q = S::LDS_Q, LDS_P = S::LDS_P;
    const DomainArgs& D = A.d[DOM];
    const DomainArgs& O = A.d[1 - DOM];
    const int tid = threadIdx.x;
    const int nx = A.nx, nz = D.nz;
    const int tx = tile % D.tiles_x, tz = tile / D.tiles_x;
    // Tiles are fixed (TX x TZ, aligned at multiples of TZ in z); a tile
    // computes its rows inside [row_lo, row_hi): tile rows [vs, ve).
    const int x0 = tx * TX;
    const int z0 = (D.row_lo / TZ + tz) * TZ;
    const int vs = max(z0, D.row_lo) - z0;
    const int ve = min(z0 + TZ, D.row_hi) - z0;
    const int ncols = min(TX, nx - x0);

    Lds<FT> L;
    L.q = (FT*)smem;
    L.p = L.q + LDS_Q;
    L.gf = (double*)(smem + (LDS_Q + LDS_P) * sizeof(FT));
    FT* ex_x = L.q;                              // [NV][TZ][TX+1]
    FT* ex_z = L.q + NV * TZ * (TX + 1);         // [NV][TZ+1][TX]

    // The interface is above this tile's last computed row (lower domain) or
    // below its first (upper domain).
    const bool has_gamma = (DOM == 0) ? (D.gamma_top && z0 + ve == nz)
                                      : (D.gamma_bot && z0 + vs == 0);

    constexpr int CZ = S::CZ;
    const int c = tid % TX;
    const int r0 = CZ * (tid / TX);
    bool okc[CZ];
#pragma unroll
    for (int h = 0; h < CZ; ++h) okc[h] = (c < ncols) && (r0 + h >= vs) && (r0 + h < ve);

    // Waves raise their issue priority while they issue the tile's global
    // loads (staging, and later the substep-base reads), so that the loads of
    // a workgroup leave early while the other workgroups of the CU compute
    // (2% per step on the 1024 x 512 workload).
    __builtin_amdgcn_s_setprio(2);

    // ---- stage the state tile (periodic in x, mirror rows beyond the domain).
    // Each thread stages its own CZ cells and, for the ring of 2 cells around
    // the tile (the two rows below it, the two rows above it, then the two
    // cells left and right of each row), ring cells tid, tid + NT, ...; all
    // its global loads are issued before any is used.  The own cells' FP64
    // values stay in registers as the stage values of the combination (FP32
    // staging).
    constexpr int NRING = HZ * HX - TX * TZ;
    constexpr int NRP = (NRING + NT - 1) / NT;   // ring positions per thread
    constexpr int NP = CZ + NRP;
    double qown[CZ][NV];
    {
        int xs[NP], zs[NP];
        bool has[NP];
#pragma unroll
        for (int h = 0; h < CZ; ++h) {
            xs[h] = c + 2;
            zs[h] = r0 + h + 2;
            has[h] = true;
        }
#pragma unroll
        for (int j = 0; j < NRP; ++j) {
            const int k = CZ + j;
            const int s = tid + j * NT;
            has[k] = s < NRING;
            const int sc = min(s, NRING - 1);
            if (sc < 2 * HX) {
                zs[k] = sc / HX;
                xs[k] = sc - zs[k] * HX;
            } else if (sc < 4 * HX) {
                const int q = sc - 2 * HX;
                zs[k] = HZ - 2 + q / HX;
                xs[k] = q - (q / HX) * HX;
            } else {
                const int q = sc - 4 * HX, jj = q & 3;
                zs[k] = 2 + (q >> 2);
                xs[k] = jj < 2 ? jj : HX - 4 + jj;
            }
        }
        double val[NP][NV];
        bool neg[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            neg[k] = false;
            if (has[k]) {
                const int col = nx > TX ? wrap1(x0 + xs[k] - 2, nx) : wrapx(x0 + xs[k] - 2, nx);
                int row = z0 + zs[k] - 2;
                if (row < 0) { row = 0; neg[k] = true; }
                else if (row >= nz) { row = nz - 1; neg[k] = true; }
                const double* src;
                size_t plane;
                if (D.use_ret && (row < D.b_lo || row >= D.b_hi)) {
                    int rr = row - D.ret_lo;
                    rr = rr < 0 ? 0 : (rr > 1 ? 1 : rr);
                    src = D.ret_in + (size_t)rr * nx + col;
                    plane = 2 * (size_t)nx;
                } else {
                    src = D.qin + (size_t)row * nx + col;
                    plane = (size_t)nz * nx;
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) val[k][v] = src[v * plane];
            }
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (has[k]) {
                const int zr = zs[k], xc = xs[k];
                FT q[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    q[v] = FT((v == 2 && neg[k]) ? -val[k][v] : val[k][v]);
                    L.q[(v * HZ + zr) * HX + xc] = q[v];
                }
                // Primitives of the tile and its 1-cell ring, from the same
                // staged values (primitive cell (zr - 1, xc - 1)).
                if (xc >= 1 && xc <= HX - 2 && zr >= 1 && zr <= HZ - 2) {
                    FT u, w, T;
                    primitives<FT>(q[0], q[1], q[2], q[3], arg_ft<FT>(A.gamma, A.gamma_f),
                                   arg_ft<FT>(A.gm1, A.gm1_f), u, w, T);
                    const int pi = (zr - 1) * PX + xc - 1;
                    L.p[pi] = u;
                    L.p[PZ * PX + pi] = w;
                    L.p[2 * PZ * PX + pi] = T;
                }
            }
        }
#pragma unroll
        for (int h = 0; h < CZ; ++h)
#pragma unroll
            for (int v = 0; v < NV; ++v) qown[h][v] = val[h][v];
    }
    // Interface flux per column, FP64, from the FP64 cell averages of the two
    // cells next to the interface (the tiles on both sides compute the same
    // bits).
    if (has_gamma && tid < TX) {
        const int col = nx > TX ? wrap1(x0 + tid, nx) : wrapx(x0 + tid, nx);
        const int own = (DOM == 0) ? nz - 1 : 0;
        const int oth = (DOM == 0) ? 0 : O.nz - 1;
        const size_t po = (size_t)nz * nx, pq = (size_t)O.nz * nx;
        const double* a = D.qin + (size_t)own * nx + col;
        const double* b = O.qin + (size_t)oth * nx + col;
        double ua, Ta, ub, Tb;
        interface_cell(a[0], a[po], a[2 * po], a[3 * po], A.gamma, A.gm1, ua, Ta);
        interface_cell(b[0], b[pq], b[2 * pq], b[3 * pq], A.gamma, A.gm1, ub, Tb);
        double f1, f3;
        if (DOM == 0) interface_flux(A, ua, Ta, ub, Tb, f1, f3);
        else interface_flux(A, ub, Tb, ua, Ta, f1, f3);
        L.gf[tid] = f1;
        L.gf[TX + tid] = f3;
    }
    __syncthreads();

    __builtin_amdgcn_s_setprio(0);

    // ---- faces: the x-face right of each of the thread's cells, the z-face
    // above it, and one edge face per thread of the first TZ + TX: the
    // x-face left of column 0 on row e (e < TZ) or the z-face below the first
    // computed row in column e - TZ.  The edge faces of both directions share
    // one pass of the face code (the direction is a per-lane value), which
    // only the first wave(s) run.
    const int re = vs - 1;
    const bool e_z = tid >= TZ;
    const int e_c = e_z ? tid - TZ : -1;
    const int e_r = e_z ? re : tid;
    const bool ex_e = e_z ? (tid - TZ < TX && tid - TZ < ncols) : (tid >= vs && tid < ve);
    const int kind_e = (e_z && z0 + vs == 0) ? FACE_BOTTOM : FACE_INTERIOR;

    // F[h]: x-face right of cell h; F[CZ + h]: z-face above it; F[2 CZ]: edge face.
    FT F[2 * CZ + 1][NV];
#pragma unroll
    for (int h = 0; h < CZ; ++h)
        if (okc[h]) face_flux<FT, S>(A, D, L, 0, c, r0 + h, FACE_INTERIOR, F[h]);
#pragma unroll
    for (int h = 0; h < CZ; ++h)
        if (okc[h]) {
            const int kind = (z0 + r0 + h == nz - 1) ? FACE_TOP : FACE_INTERIOR;
            face_flux<FT, S>(A, D, L, 1, c, r0 + h, kind, F[CZ + h]);
        }
    if (ex_e) face_flux<FT, S>(A, D, L, e_z ? 1 : 0, e_c, e_r, kind_e, F[2 * CZ]);

    __builtin_amdgcn_s_setprio(2);
    // The stage value of the combination (staged FP64 registers, or the FP64
    // tile) and the pointwise read of the substep base U, which completes
    // while the fluxes are exchanged.
    const int col = x0 + c;
    const size_t plane = (size_t)nz * nx;
    const size_t nbx = (size_t)(D.b_hi - D.b_lo) * nx;
    double qc[CZ][NV], Ub[CZ][NV];
#pragma unroll
    for (int h = 0; h < CZ; ++h) {
        const int row = z0 + r0 + h;
        const bool ok = okc[h];
        const bool inb = (row >= D.b_lo && row < D.b_hi);
        const Combine cb = pick_combine(D.buf, D.main, inb);
        const size_t id = (size_t)row * nx + col;
        // The stage value: the staged FP64 value itself (own rows that are
        // computed are never mirror rows, nor taken from the retained rows).
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Ub[h][v] = 0.0;
            qc[h][v] = sizeof(FT) == 8 ? (double)L.q[qidx<S>(v, r0 + h, c)] : qown[h][v];
        }
        if (ok && cb.mode != MODE_RHS && cb.alpha != 0.0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Ub[h][v] = D.base[v * plane + id];
        }
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();   // all LDS reads of the staged state are done

    // Fluxes back from the face-normal frame to (rho, rho u, rho w, rho E).
    auto put_x = [&](int cc, int rr, const FT* f) {
        FT* e = ex_x + rr * (TX + 1) + cc + 1;
        constexpr int st = TZ * (TX + 1);
        e[0] = f[0]; e[st] = f[1]; e[2 * st] = f[2]; e[3 * st] = f[3];
    };
    auto put_z = [&](int cc, int rr, const FT* f) {
        FT* e = ex_z + (rr + 1) * TX + cc;
        constexpr int st = (TZ + 1) * TX;
        e[0] = f[0]; e[st] = f[2]; e[2 * st] = f[1]; e[3 * st] = f[3];
    };
#pragma unroll
    for (int h = 0; h < CZ; ++h)
        if (okc[h]) { put_x(c, r0 + h, F[h]); put_z(c, r0 + h, F[CZ + h]); }
    if (ex_e) {
        if (e_z) put_z(e_c, re, F[2 * CZ]);
        else put_x(-1, tid, F[2 * CZ]);
    }
    __syncthreads();

    // ---- divergence (FP64: differences of two face fluxes are exact for FP32
    // fluxes, so the exchange stays conservative), source and stage
    // combination.
#pragma unroll
    for (int h = 0; h < CZ; ++h) {
        const bool ok = okc[h];
        if (!ok) continue;
        const int r = r0 + h;
        const int row = z0 + r;
        double R[NV];
        // The right x-face and the top z-face are this thread's own (still in
        // registers; the z-face in its normal frame); the left and bottom
        // ones come from the exchange.
        constexpr int zmap[NV] = {0, 2, 1, 3};
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const FT* fx = ex_x + v * TZ * (TX + 1) + r * (TX + 1) + c;
            const FT* fz = ex_z + v * (TZ + 1) * TX + r * TX + c;
            R[v] = -((double)F[h][v] - (double)fx[0]) * A.hinv_dx -
                   ((double)F[CZ + h][zmap[v]] - (double)fz[0]) * D.hinv_dz;
        }
        // Interface viscous flux (FP64, same bits on both sides): it leaves the
        // lower domain through its top face and enters the upper domain
        // through its bottom face.
        if (DOM == 0 && D.gamma_top && row == nz - 1) {
            R[1] += L.gf[c] * D.inv_dz;
            R[3] += L.gf[TX + c] * D.inv_dz;
        }
        if (DOM == 1 && D.gamma_bot && row == 0) {
            R[1] -= L.gf[c] * D.inv_dz;
            R[3] -= L.gf[TX + c] * D.inv_dz;
        }
        R[2] += qc[h][0] * A.gravity;
        R[3] += qc[h][2] * A.gravity;

        const bool inb = (row >= D.b_lo && row < D.b_hi);
        const Combine cb = pick_combine(D.buf, D.main, inb);
        const size_t id = (size_t)row * nx + col;
        if (cb.mode == MODE_RHS) {
#pragma unroll
            for (int v = 0; v < NV; ++v) st_dev(A.dev_stores != 0, &D.out[v * plane + id], R[v]);
        } else if (cb.alpha == 0.0) {
            // First stage of a base step: Qin is the base U itself.
#pragma unroll
            for (int v = 0; v < NV; ++v) st_dev(A.dev_stores != 0, &D.out[v * plane + id], qc[h][v] + cb.bh * R[v]);
        } else {
            // Increment form of alpha U + beta (Qin + h R): U + beta (Qin - U)
            // + beta h R, exact when R = 0 and Qin = U.
            double inc[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) inc[v] = cb.beta * (qc[h][v] - Ub[h][v]) + cb.bh * R[v];
            if (cb.mode == MODE_STAGE) {
#pragma unroll
                for (int v = 0; v < NV; ++v) st_dev(A.dev_stores != 0, &D.out[v * plane + id], Ub[h][v] + inc[v]);
            } else {
                // Buffer: accumulate the increments of the m trial steps and
                // add their mean to q^B_n after the last one.
                const size_t ia = (size_t)(row - D.b_lo) * nx + col;
                if (cb.mode == MODE_ACC_FIRST) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) st_dev(A.dev_stores != 0, &D.acc[v * nbx + ia], inc[v]);
                } else if (cb.mode == MODE_ACC_ADD) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) st_dev(A.dev_stores != 0, &D.acc[v * nbx + ia], D.acc[v * nbx + ia] + inc[v]);
                } else {
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        st_dev(A.dev_stores != 0, &D.out[v * plane + id], Ub[h][v] + (D.acc[v * nbx + ia] + inc[v]) * A.inv_m);
                }
            }
        }
        if (D.ret_out && row >= D.ret_lo && row < D.ret_lo + 2) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                st_dev(A.dev_stores != 0, &D.ret_out[(size_t)(v * 2 + row - D.ret_lo) * nx + col], qc[h][v]);
        }
    }
}

#ifndef MPRK_WAVES_PER_EU
#define MPRK_WAVES_PER_EU 3
#endif

// Tiles of one stage record, block b of its nblocks: domain A.first takes the
// first blocks (the host puts the domain with the shorter tiles first so
// they do not form a tail).
template <class FT, class S>
__device__ __forceinline__ void record_block(const StageArgs& A, int b, bool remap, char* smem)
{
    const int n0 = A.d[A.first].ntiles;
    const int dom = (b < n0) ? A.first : 1 - A.first;
    int t = (b < n0) ? b : b - n0;
    // The second domain's blocks keep j % 8 == XCD only if n0 % 8 == 0.
    if (remap && (b < n0 || (n0 % 8) == 0)) t = xcd_contiguous(t, (b < n0) ? n0 : A.nblocks - n0);
    if (dom == 0) stage_tile<0, FT, S>(A, t, smem);
    else stage_tile<1, FT, S>(A, t, smem);
}

template <class FT, class S>
__global__ __launch_bounds__(S::NT) __attribute__((amdgpu_waves_per_eu(MPRK_WAVES_PER_EU)))
void stage_kernel(const StageArgs A)
{
    __shared__ __align__(16) char smem[S::template lds_bytes<FT>()];
    record_block<FT, S>(A, blockIdx.x, true, smem);
}

// One launch over several stage records (batched members): blocks are
// remapped so that each XCD takes a contiguous range, then look up their
// range's stage record in the per-block map (one uniform load; a binary
// search over the ranges took a chain of dependent loads per workgroup).
template <class FT, class S>
__global__ __launch_bounds__(S::NT) __attribute__((amdgpu_waves_per_eu(MPRK_WAVES_PER_EU)))
void batch_kernel(const StageArgs* __restrict__ tab, const BatchEntry* __restrict__ bmap, int nblocks)
{
    __shared__ __align__(16) char smem[S::template lds_bytes<FT>()];
    const int b = xcd_contiguous(blockIdx.x, nblocks);
    const BatchEntry e = bmap[b];
    record_block<FT, S>(tab[e.arg], b - e.begin, false, smem);
}

// ---------------------------------------------------------------------------
// Persistent dataflow kernel.
// ---------------------------------------------------------------------------
// Wait until every tile this task reads has finished stage g - 1: the eight
// neighbours (x periodic) and, next to the interface, the tile across it.
// Called by the whole of wave 0: lane l < 9 polls neighbour (l%3 - 1, l/3 - 1),
// lane 9 the interface partner, all in parallel; a wave-wide vote decides.
// Returns false once the launch has run longer than its limit (counted from
// t_start, this workgroup's start, which for a cooperative launch is the
// launch's start) or another workgroup has aborted; the kernel then exits
// without finishing.  The limit is on the whole launch, not on each wait, so
// however many waits a workgroup makes, it exits within the limit plus one
// tile's work.
__device__ bool wait_inputs(const PersistArgs& P, const MemberRun& M, const TileRef& tr, int g,
                            int64_t t_start)
{
    const int need = g - 1;
    if (need <= 0) return true;
    const int lane = threadIdx.x & 63;
    const int tzmax = M.tiles_z[tr.dom] - 1;
    int dep = -1;
    if (lane < 9 && lane != 4) {
        const int dx = lane % 3 - 1, dz = lane / 3 - 1;
        const int tz = tr.tz + dz;
        int tx = tr.tx + dx;
        tx = tx < 0 ? tx + M.tiles_x : (tx >= M.tiles_x ? tx - M.tiles_x : tx);
        if (tz >= 0 && tz <= tzmax && !(tx == tr.tx && tz == tr.tz))
            dep = M.done_base[tr.dom] + tz * M.tiles_x + tx;
    } else if (lane == 9) {
        if (tr.dom == 0 && tr.tz == tzmax) dep = M.done_base[1] + tr.tx;
        if (tr.dom == 1 && tr.tz == 0) dep = M.done_base[0] + (M.tiles_z[0] - 1) * M.tiles_x + tr.tx;
    }
    while (true) {
        const bool ready = dep < 0 ||
            __hip_atomic_load(P.done + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        if (__all(ready)) break;
        __builtin_amdgcn_s_sleep(1);
        const bool ab = lane == 0 &&
            __hip_atomic_load(P.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        if (__any(ab) || wall_clock64() - t_start > P.run_ticks) {
            if (lane == 0) __hip_atomic_store(P.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    // Make the producers' stores visible to this workgroup's loads.
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

#ifndef MPRK_PERSIST_WAVES_PER_EU
#define MPRK_PERSIST_WAVES_PER_EU 2
#endif

template <class FT, class S>
__global__ __launch_bounds__(S::NT) __attribute__((amdgpu_waves_per_eu(MPRK_PERSIST_WAVES_PER_EU)))
void persistent_kernel(const PersistArgs P)
{
    __shared__ __align__(16) char smem[S::template lds_bytes<FT>()];
    __shared__ int s_go;
    const int64_t t_start = wall_clock64();
    const int G = gridDim.x;
    for (int g = 1; g <= P.gmax; ++g) {
        // Blocks j and j + G run on the same XCD when G % 8 == 0; the remap
        // gives each XCD a contiguous range of tiles.
        for (int i = blockIdx.x; i < P.ntiles; i += G) {
            const int t = (G % 8 == 0) ? xcd_contiguous(i, P.ntiles) : i;
            const TileRef tr = P.tiles[t];
            const MemberRun& M = P.members[tr.member];
            const int step = (g - 1) / M.nslots, slot = (g - 1) - step * M.nslots;
            const int rec = step >= M.nsteps ? -1 : (M.slot_stage ? M.slot_stage[slot] : slot);
            const StageArgs& A = M.stages[rec < 0 ? 0 : rec];
            const DomainArgs& D = A.d[tr.dom];
            const int z0 = tr.tz * S::TZ;
            const bool work = rec >= 0 && D.row_hi > D.row_lo && z0 < D.row_hi && z0 + S::TZ > D.row_lo;
            if (work) {
                if (threadIdx.x < 64) {
                    const bool ok = wait_inputs(P, M, tr, g, t_start);
                    if (threadIdx.x == 0) s_go = ok ? 1 : 0;
                }
                __syncthreads();
                if (!s_go) return;
                const int rel = (tr.tz - D.row_lo / S::TZ) * D.tiles_x + tr.tx;
                if (tr.dom == 0) stage_tile<0, FT, S>(A, rel, smem);
                else stage_tile<1, FT, S>(A, rel, smem);
                // Every wave's stores are complete before thread 0 publishes.
                __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(P.done + M.done_base[tr.dom] + tr.tz * M.tiles_x + tr.tx, g,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

__global__ void fill_i32(int32_t* p, int32_t v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Reductions.
// ---------------------------------------------------------------------------
constexpr int RV = 5;        // components summed (2D uses the first 4)

struct RedVal {
    double s[RV], e[RV];     // compensated sums: value + error term
    double lam, cour, vis, bad;
};

__device__ __forceinline__ void two_sum(double& s, double& e, double x)
{
    const double t = s + x;
    e += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

__device__ __forceinline__ void red_combine(RedVal& a, const RedVal& b)
{
#pragma unroll
    for (int v = 0; v < RV; ++v) {
        two_sum(a.s[v], a.e[v], b.s[v]);
        a.e[v] += b.e[v];
    }
    a.lam = fmax(a.lam, b.lam);
    a.cour = fmax(a.cour, b.cour);
    a.vis = fmax(a.vis, b.vis);
    a.bad = fmax(a.bad, b.bad);
}

// Field layout: sums [0, 5), compensation terms [5, 10), then lambda,
// courant, visc, bad.
__device__ __forceinline__ void red_store(double* p, const RedVal& a)
{
#pragma unroll
    for (int v = 0; v < RV; ++v) { p[v] = a.s[v]; p[RV + v] = a.e[v]; }
    p[10] = a.lam; p[11] = a.cour; p[12] = a.vis; p[13] = a.bad;
}

__device__ __forceinline__ void red_load(const double* p, RedVal& a)
{
#pragma unroll
    for (int v = 0; v < RV; ++v) { a.s[v] = p[v]; a.e[v] = p[RV + v]; }
    a.lam = p[10]; a.cour = p[11]; a.vis = p[12]; a.bad = p[13];
}

// Fixed-shape tree over the block: the result does not depend on timing.
__device__ void block_tree(RedVal& mine, double* sh)
{
    const int tid = threadIdx.x;
    red_store(sh + tid * RED_FIELDS, mine);
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) {
            RedVal a, b;
            red_load(sh + tid * RED_FIELDS, a);
            red_load(sh + (tid + s) * RED_FIELDS, b);
            red_combine(a, b);
            red_store(sh + tid * RED_FIELDS, a);
        }
        __syncthreads();
    }
    red_load(sh, mine);
}

// Totals, stability measures and the bad-state flag of one domain (2D: the
// components are (rho, rho u, rho w, rho E); 3D: (rho, rho u, rho v, rho w,
// rho E)).
__device__ __forceinline__ void reduce_partial_body(const ReduceArgs& A, int dom, int blk, double* sh)
{
    const double* q = A.q[dom];
    const int nv = A.nv;
    const bool three = nv == 5;
    const int n = A.nz[dom] * A.ny * A.nx;
    const double inv_dz = A.inv_dz[dom], vc = A.visc_coef[dom];
    RedVal m;
#pragma unroll
    for (int v = 0; v < RV; ++v) { m.s[v] = 0.0; m.e[v] = 0.0; }
    m.lam = m.cour = m.vis = m.bad = 0.0;
    for (int i = blk * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) {
        double c[RV];
#pragma unroll
        for (int v = 0; v < RV; ++v) c[v] = v < nv ? q[(size_t)v * n + i] : 0.0;
#pragma unroll
        for (int v = 0; v < RV; ++v) two_sum(m.s[v], m.e[v], c[v]);
        const double rho = c[0];
        const double mx = c[1], my = three ? c[2] : 0.0, mz = three ? c[3] : c[2];
        const double en = three ? c[4] : c[3];
        const double ir = 1.0 / rho;
        const double u = mx * ir, v = my * ir, w = mz * ir;
        const double p = A.gm1 * (en - 0.5 * (mx * u + my * v + mz * w));
        bool ok = (rho > 0.0) && (p > 0.0);
#pragma unroll
        for (int k = 0; k < RV; ++k) ok = ok && isfinite(c[k]);
        if (!ok) {
            m.bad = 1.0;
        } else {
            const double a = sqrt(A.gamma * p * ir);
            const double sx = (fabs(u) + a) * A.inv_dx;
            const double sy = three ? (fabs(v) + a) * A.inv_dy : 0.0;
            const double sz = (fabs(w) + a) * inv_dz;
            m.lam = fmax(m.lam, sx + sy + sz);
            m.cour = fmax(m.cour, fmax(fmax(sx, sy), sz));
            m.vis = fmax(m.vis, vc * ir);
        }
    }
    block_tree(m, sh);
    if (threadIdx.x == 0) red_store(A.partial + ((size_t)dom * RED_BLOCKS + blk) * RED_FIELDS, m);
}

__device__ __forceinline__ void reduce_final_body(const ReduceArgs& A, int dom, double* sh)
{
    static_assert(RED_BLOCKS == RED_THREADS, "one partial per thread");
    RedVal m;
    red_load(A.partial + ((size_t)dom * RED_BLOCKS + threadIdx.x) * RED_FIELDS, m);
    block_tree(m, sh);
    if (threadIdx.x == 0) red_store(A.final_ + (size_t)dom * RED_FIELDS, m);
}

__global__ __launch_bounds__(RED_THREADS) void reduce_partial(const ReduceArgs A)
{
    __shared__ double sh[RED_THREADS * RED_FIELDS];
    reduce_partial_body(A, blockIdx.y, blockIdx.x, sh);
}

__global__ __launch_bounds__(RED_THREADS) void reduce_final(const ReduceArgs A)
{
    __shared__ double sh[RED_THREADS * RED_FIELDS];
    reduce_final_body(A, blockIdx.x, sh);
}

// Every member of a batch at once: blockIdx.z (partial) / blockIdx.y (final)
// selects the member's record.
__global__ __launch_bounds__(RED_THREADS) void reduce_partial_batch(const ReduceArgs* __restrict__ tab)
{
    __shared__ double sh[RED_THREADS * RED_FIELDS];
    reduce_partial_body(tab[blockIdx.z], blockIdx.y, blockIdx.x, sh);
}

__global__ __launch_bounds__(RED_THREADS) void reduce_final_batch(const ReduceArgs* __restrict__ tab)
{
    __shared__ double sh[RED_THREADS * RED_FIELDS];
    reduce_final_body(tab[blockIdx.y], blockIdx.x, sh);
}

using S0 = Shape<32, 16>;
using S1 = Shape<16, 32>;
using S2 = Shape<64, 8>;
using S3 = Shape<32, 8>;

// The host's view of each shape (tile counts) must match the kernels'.
template <class S>
constexpr bool same_dims(int shape)
{
    return tile_dims(shape).tx == S::TX && tile_dims(shape).tz == S::TZ && tile_dims(shape).nt == S::NT;
}
static_assert(same_dims<S0>(TILE_32x16) && same_dims<S1>(TILE_16x32) && same_dims<S2>(TILE_64x8) &&
                  same_dims<S3>(TILE_32x8),
              "tile shape table");

// Calls f.template operator()<FT, S>() for the flux type and shape.
template <class F>
auto with_kernel(bool flux32, int shape, F&& f)
{
    switch (shape) {
    case TILE_16x32: return flux32 ? f.template operator()<float, S1>() : f.template operator()<double, S1>();
    case TILE_64x8: return flux32 ? f.template operator()<float, S2>() : f.template operator()<double, S2>();
    case TILE_32x8: return flux32 ? f.template operator()<float, S3>() : f.template operator()<double, S3>();
    default: return flux32 ? f.template operator()<float, S0>() : f.template operator()<double, S0>();
    }
}

}  // namespace

hipError_t launch_stage(const StageArgs& a, int shape, hipStream_t s)
{
    if (a.nblocks <= 0) return hipSuccess;
    return with_kernel(a.flux32 != 0, shape, [&]<class FT, class S>() {
        hipLaunchKernelGGL((stage_kernel<FT, S>), dim3(a.nblocks), dim3(S::NT), 0, s, a);
        return hipGetLastError();
    });
}

KernelRef stage_kernel_ref(bool flux32, int shape)
{
    return with_kernel(flux32, shape, []<class FT, class S>() {
        return KernelRef{(const void*)stage_kernel<FT, S>, S::NT};
    });
}

hipError_t launch_batch(const StageArgs* tab, const BatchEntry* bmap, int nblocks, bool flux32, int shape,
                        hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    return with_kernel(flux32, shape, [&]<class FT, class S>() {
        hipLaunchKernelGGL((batch_kernel<FT, S>), dim3(nblocks), dim3(S::NT), 0, s, tab, bmap, nblocks);
        return hipGetLastError();
    });
}

KernelRef batch_kernel_ref(bool flux32, int shape)
{
    return with_kernel(flux32, shape, []<class FT, class S>() {
        return KernelRef{(const void*)batch_kernel<FT, S>, S::NT};
    });
}

hipError_t launch_persistent(const PersistArgs& a, int grid, bool flux32, int shape, hipStream_t s)
{
    return with_kernel(flux32, shape, [&]<class FT, class S>() {
        void* args[] = {(void*)&a};
        return hipLaunchCooperativeKernel((const void*)persistent_kernel<FT, S>, dim3(grid), dim3(S::NT),
                                          args, 0, s);
    });
}

int persistent_blocks_per_cu(bool flux32, int shape)
{
    return with_kernel(flux32, shape, []<class FT, class S>() {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)persistent_kernel<FT, S>, S::NT,
                                                         0) != hipSuccess)
            return 0;
        return nb;
    });
}

hipError_t launch_fill_i32(int32_t* p, int32_t value, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_reduce_batch(const ReduceArgs* tab, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_partial_batch, dim3(RED_BLOCKS, 2, n), dim3(RED_THREADS), 0, s, tab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_batch, dim3(2, n), dim3(RED_THREADS), 0, s, tab);
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_partial, dim3(RED_BLOCKS, 2), dim3(RED_THREADS), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final, dim3(2), dim3(RED_THREADS), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reduction scratch of the allocation-free diagnostics entry point: the
// partial results of reduce_partial ([2][RED_BLOCKS][RED_FIELDS]) followed by
// the final fields ([2][RED_FIELDS]).  One copy per device, held until the
// process ends; every call on a device shares it.  reduce_partial writes
// every partial slot before reduce_final reads it, so nothing needs clearing
// between calls.
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];

namespace {
constexpr int STATIC_SCRATCH_MAX_DEVICES = 64;
std::mutex static_scratch_mu;
double* static_scratch_ptr[STATIC_SCRATCH_MAX_DEVICES];
}  // namespace

// Device address of the scratch array on the current device.  The name
// `scratch` is a host-side stand-in in host code, so the address is looked up
// (once per device, with that device current) and kept.
hipError_t static_scratch_address(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= STATIC_SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(static_scratch_mu);
    if (!static_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        static_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = static_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace mprk
