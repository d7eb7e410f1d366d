// mprk_kernels.hip -- gfx950 kernels of the MPRK library.
//
// stage_kernel: one MPRK stage for every cell a launch covers, in both
// domains at once.  For each cell: the coupled finite-volume RHS (Section 2.1,
// Appendix B restricted to x-z; local Lax-Friedrichs flux with Roe-average
// wave speed, common-value viscous flux, bulk-coefficient interface flux of
// eq. bulk-flux) and the stage combination of its partition (eq. MRK2 in a
// low-storage substep form).
//
// Tiling: a workgroup of 256 threads owns a 32 x 16 tile of one domain.  The
// tile's conserved state (2-cell halo) and primitives u, w, T (1-cell halo)
// are staged in LDS; every face of the tile is computed exactly once (two
// faces per cell plus one left column and one bottom row of edge faces) by a
// single direction-generic face routine; the fluxes are exchanged through LDS
// (aliasing the staged state) and each thread forms the divergence of its
// two cells.
//
// reduce_*: deterministic (fixed-order) device reductions for the totals,
// stability measures and the physical-state flag.
#include "mprk_internal.h"

namespace mprk {

namespace {

#ifndef MPRK_FACE_PAIRS
#define MPRK_FACE_PAIRS 0
#endif
// Keep face evaluations from being interleaved by the scheduler: the
// interleaved form needs far more registers than the occupancy allows.
#ifndef MPRK_FACE_SEQ
#define MPRK_FACE_SEQ 0
#endif
#if MPRK_FACE_SEQ
#define FACE_SCHED_BARRIER() __builtin_amdgcn_sched_barrier(0)
#else
#define FACE_SCHED_BARRIER() ((void)0)
#endif

constexpr int LDS_Q = NV * HZ * HX;        // staged conserved state
constexpr int LDS_P = 3 * PZ * PX;         // staged primitives u, w, T
constexpr int LDS_G = 2 * TX;              // u, T of the cell across the interface
constexpr int LDS_O = NV * TX;             // conserved state of that cell
constexpr int LDS_EX = NV * TZ * (TX + 1) + NV * (TZ + 1) * TX;  // face fluxes
constexpr int LDS_N = LDS_Q + LDS_P + LDS_G + LDS_O;
static_assert(LDS_EX <= LDS_Q + LDS_P, "flux exchange must fit in the staged state");
constexpr int LOAD_RG = NT / HX;                        // row groups of the loader
constexpr int LOAD_THREADS = LOAD_RG * HX;
constexpr int LOAD_ROWS = (HZ + LOAD_RG - 1) / LOAD_RG; // rows per loader thread

__device__ __forceinline__ int wrapx(int c, int nx)
{
    int r = c % nx;
    return r < 0 ? r + nx : r;
}

// 1/sqrt(x) for positive normal x: hardware estimate refined by two Newton
// steps y <- y + y (1 - x y^2) / 2 (quadratic convergence; a few ulp).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double r = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, r, y);
    r = fma(-(x * y), y, 1.0);
    return fma(0.5 * y, r, y);
}

// sqrt(x) = x / sqrt(x) for positive normal x (no scaling for subnormals,
// zero or infinity, which a physical state never produces; a non-physical
// one yields NaN, which the device status check reports).
__device__ __forceinline__ double sqrt_nr(double x) { return x * rsqrt_nr(x); }

// 1/x for positive normal x: hardware estimate refined by two Newton steps
// y <- y + y (1 - x y).
__device__ __forceinline__ double rcp_nr(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// Cell primitives.  Contraction is off so that the value is identical
// wherever it is evaluated: the interface flux is computed on both sides of
// the interface and must agree to the bit for conservation.
__device__ __forceinline__ void primitives(double rho, double mx, double mz, double en,
                                           double gamma, double gm1, double& u, double& w,
                                           double& T)
{
#pragma clang fp contract(off)
    const double ir = rcp_nr(rho);
    u = mx * ir;
    w = mz * ir;
    double p = gm1 * (en - 0.5 * (mx * u + mz * w));
    T = gamma * p * ir;
}

// Interface viscous flux in +z (Appendix B, eq. bulk-flux; hat w = 0 and
// hat sigma_zz = 0 on the lid): (0, sigma_xz, 0, u_w sigma_xz - Pi_z) with
// sigma_xz = b_u (u2 - u1), Pi_z = -b_T (T2 - T1), u_w = u1 + sigma dz1/(2 mu1).
// Index 1 is the lower cell, 2 the upper cell.  Contraction off: both domains
// evaluate it and must obtain the same bits.
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

struct Lds {
    double* q;   // [NV][HZ][HX]
    double* p;   // [3][PZ][PX]
    double* g;   // [2][TX]
    double* o;   // [NV][TX]
};

__device__ __forceinline__ int qidx(int v, int r, int c) { return (v * HZ + r + 2) * HX + c + 2; }
__device__ __forceinline__ int pidx(int f, int r, int c) { return (f * PZ + r + 1) * PX + c + 1; }

// Boundary kinds of a face.
enum : int { FACE_INTERIOR = 0, FACE_TOP = 1, FACE_BOTTOM = 2 };

// Numerical flux (inviscid minus viscous) through the face between tile cell
// (c, r) and its +dir neighbour, in the face-normal frame: returns
// (F_rho, F_normal-momentum, F_tangential-momentum, F_energy).
//   kind FACE_TOP:    (c, r) is the top interior row; the other side is its
//                     mirror; gam = interface above.
//   kind FACE_BOTTOM: (c, r+1) is the bottom interior row; gam = interface
//                     below.
// For a wall the viscous flux is zero; at the interface it is the bulk flux.
// N independent faces are evaluated in lockstep so that their dependency
// chains interleave.
template <int DOM, int dir, int N>
__device__ __forceinline__ void face_fluxes(const StageArgs& A, const DomainArgs& D, const Lds& L,
                                            const int (&c)[N], const int (&r)[N],
                                            const int (&kind)[N], double (&F)[N][NV])
{
    const double gamma = A.gamma, gm1 = A.gm1;
    constexpr int sn = dir ? HX : 1;         // normal stride in the state tile
    constexpr int vn = dir ? 2 : 1;          // normal momentum component
    constexpr int vt = dir ? 1 : 2;          // tangential momentum component
    constexpr int plane = HZ * HX;
    constexpr int comp[NV] = {0, vn, vt, 3};

    // Reconstruction of conserved variables with central cell gradients:
    // qL = q_c + (q_{c+1} - q_{c-1})/4, qR = q_{c+1} - (q_{c+2} - q_c)/4.
    double qL[N][NV], qR[N][NV];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const int base = qidx(0, r[n], c[n]);
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double* s = L.q + comp[k] * plane + base;
            const double qm = s[-sn], q0 = s[0], q1 = s[sn], q2 = s[2 * sn];
            qL[n][k] = q0 + 0.25 * (q1 - qm);
            qR[n][k] = q1 - 0.25 * (q2 - q0);
        }
        if (kind[n] == FACE_TOP) {
            qR[n][0] = qL[n][0]; qR[n][1] = -qL[n][1]; qR[n][2] = qL[n][2]; qR[n][3] = qL[n][3];
        } else if (kind[n] == FACE_BOTTOM) {
            qL[n][0] = qR[n][0]; qL[n][1] = -qR[n][1]; qL[n][2] = qR[n][2]; qL[n][3] = qR[n][3];
        }
    }

    // Local Lax-Friedrichs flux, lambda = max(|u_n| + a) over qL, qR and the
    // Roe average (sqrt(rho)-weighted velocity and total enthalpy).  One
    // reciprocal square root per side gives 1/rho and sqrt(rho).
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const double* l = qL[n];
        const double* q = qR[n];
        const double yL = rsqrt_nr(l[0]), yR = rsqrt_nr(q[0]);
        const double rL = yL * yL, rR = yR * yR;
        const double sL = l[0] * yL, sR = q[0] * yR;
        const double unL = l[1] * rL, utL = l[2] * rL;
        const double unR = q[1] * rR, utR = q[2] * rR;
        const double pL = gm1 * (l[3] - 0.5 * (l[1] * unL + l[2] * utL));
        const double pR = gm1 * (q[3] - 0.5 * (q[1] * unR + q[2] * utR));
        const double aL = sqrt_nr(gamma * pL * rL);
        const double aR = sqrt_nr(gamma * pR * rR);
        const double iw = rcp_nr(sL + sR);
        const double unr = (sL * unL + sR * unR) * iw;
        const double utr = (sL * utL + sR * utR) * iw;
        const double HL = (l[3] + pL) * rL, HR = (q[3] + pR) * rR;
        const double Hr = (sL * HL + sR * HR) * iw;
        const double ar = sqrt_nr(gm1 * (Hr - 0.5 * (unr * unr + utr * utr)));
        const double lam = fmax(fmax(fabs(unL) + aL, fabs(unR) + aR), fabs(unr) + ar);
        const double hl = 0.5 * lam;
        F[n][0] = 0.5 * (l[1] + q[1]) - hl * (q[0] - l[0]);
        F[n][1] = 0.5 * (l[1] * unL + q[1] * unR + pL + pR) - hl * (q[1] - l[1]);
        F[n][2] = 0.5 * (l[2] * unL + q[2] * unR) - hl * (q[2] - l[2]);
        F[n][3] = 0.5 * ((l[3] + pL) * unL + (q[3] + pR) * unR) - hl * (q[3] - l[3]);
    }

#pragma unroll
    for (int n = 0; n < N; ++n) {
        if (kind[n] == FACE_INTERIOR) {
            // Common values: averaged velocity, normal derivative by finite
            // difference, tangential derivative by averaging cell gradients.
            const int pb = pidx(0, r[n], c[n]);
            constexpr int pn = dir ? PX : 1;
            constexpr int pt = dir ? 1 : PX;
            constexpr int fn = dir ? 1 : 0;  // normal velocity in the primitive tile
            constexpr int ft = dir ? 0 : 1;
            constexpr int pp = PZ * PX;
            const double* Un = L.p + fn * pp + pb;
            const double* Ut = L.p + ft * pp + pb;
            const double* Tt = L.p + 2 * pp + pb;
            const double inv_n = dir ? D.inv_dz : A.inv_dx;
            const double inv_t4 = 0.25 * (dir ? A.inv_dx : D.inv_dz);
            const double unA = Un[0], unB = Un[pn], utA = Ut[0], utB = Ut[pn];
            const double dn_un = (unB - unA) * inv_n;
            const double dn_ut = (utB - utA) * inv_n;
            const double dn_T = (Tt[pn] - Tt[0]) * inv_n;
            const double dt_un = (Un[pt] - Un[-pt] + Un[pn + pt] - Un[pn - pt]) * inv_t4;
            const double dt_ut = (Ut[pt] - Ut[-pt] + Ut[pn + pt] - Ut[pn - pt]) * inv_t4;
            const double mu = D.mu;
            const double snn = mu * ((4.0 / 3.0) * dn_un - (2.0 / 3.0) * dt_ut);
            const double snt = mu * (dn_ut + dt_un);
            F[n][1] -= snn;
            F[n][2] -= snt;
            F[n][3] -= 0.5 * (unA + unB) * snn + 0.5 * (utA + utB) * snt + D.kappa * dn_T;
        } else {
            const bool gam = (kind[n] == FACE_TOP) ? D.gamma_top : D.gamma_bot;
            if (gam) {
                // Only z-faces reach here: normal = w, tangential = u.
                double u1, T1, u2, T2;
                if (DOM == 0) {   // interface above the lower domain's top row r
                    u1 = L.p[pidx(0, r[n], c[n])];
                    T1 = L.p[pidx(2, r[n], c[n])];
                    u2 = L.g[c[n]];
                    T2 = L.g[TX + c[n]];
                } else {          // interface below the upper domain's bottom row r+1
                    u1 = L.g[c[n]];
                    T1 = L.g[TX + c[n]];
                    u2 = L.p[pidx(0, r[n] + 1, c[n])];
                    T2 = L.p[pidx(2, r[n] + 1, c[n])];
                }
                double f1, f3;
                interface_flux(A, u1, T1, u2, T2, f1, f3);
                F[n][2] -= f1;   // tangential momentum (x) component
                F[n][3] -= f3;
            }
        }
    }
}

template <int DOM>
__device__ void stage_tile(const StageArgs& A, int tile, double* lds)
{
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

    Lds L;
    L.q = lds;
    L.p = lds + LDS_Q;
    L.g = L.p + LDS_P;
    L.o = L.g + LDS_G;
    double* ex_x = lds;                          // [NV][TZ][TX+1]
    double* ex_z = lds + NV * TZ * (TX + 1);     // [NV][TZ+1][TX]

    const bool has_gamma = (DOM == 0) ? (D.gamma_top && z0 + ve == nz)
                                      : (D.gamma_bot && z0 + vs == 0);

    const int c = tid % TX;
    const int r0 = 2 * (tid / TX);
    const bool ok0 = (c < ncols) && (r0 >= vs) && (r0 < ve);
    const bool ok1 = (c < ncols) && (r0 + 1 >= vs) && (r0 + 1 < ve);

    // ---- stage the state tile (periodic in x, mirror rows beyond the domain).
    // Each of LOAD_THREADS threads owns one tile column and LOAD_ROWS rows
    // (stride LOAD_RG); all its global loads are issued before any is used.
    if (tid < LOAD_THREADS) {
        const int xc = tid % HX, rg = tid / HX;
        const int col = wrapx(x0 + xc - 2, nx);
        double val[LOAD_ROWS][NV];
        bool neg[LOAD_ROWS];
#pragma unroll
        for (int k = 0; k < LOAD_ROWS; ++k) {
            const int zr = rg + LOAD_RG * k;
            neg[k] = false;
            if (zr < HZ) {
                int row = z0 + zr - 2;
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
        for (int k = 0; k < LOAD_ROWS; ++k) {
            const int zr = rg + LOAD_RG * k;
            if (zr < HZ) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    L.q[(v * HZ + zr) * HX + xc] = (v == 2 && neg[k]) ? -val[k][v] : val[k][v];
            }
        }
    }
    if (has_gamma) {
        const int orow = (DOM == 0) ? 0 : O.nz - 1;
        for (int i = tid; i < NV * TX; i += NT) {
            const int v = i / TX, c = i - v * TX;
            const int col = wrapx(x0 + c, nx);
            L.o[i] = O.qin[((size_t)v * O.nz + orow) * nx + col];
        }
    }
    __syncthreads();

    // ---- primitives on the tile plus a 1-cell ring
    for (int idx = tid; idx < PZ * PX; idx += NT) {
        const int pr = idx / PX, pc = idx - pr * PX;
        const int b = qidx(0, pr - 1, pc - 1);
        double u, w, T;
        primitives(L.q[b], L.q[b + HZ * HX], L.q[b + 2 * HZ * HX], L.q[b + 3 * HZ * HX],
                   A.gamma, A.gm1, u, w, T);
        L.p[idx] = u;
        L.p[PZ * PX + idx] = w;
        L.p[2 * PZ * PX + idx] = T;
    }
    if (has_gamma && tid < TX) {
        double u, w, T;
        primitives(L.o[tid], L.o[TX + tid], L.o[2 * TX + tid], L.o[3 * TX + tid], A.gamma,
                   A.gm1, u, w, T);
        L.g[tid] = u;
        L.g[TX + tid] = T;
    }
    __syncthreads();

    // ---- faces

    double qc[2][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        qc[0][v] = L.q[qidx(v, r0, c)];
        qc[1][v] = L.q[qidx(v, r0 + 1, c)];
    }

    // Slots 0,1: x-faces right of the two cells; 2,3: z-faces above them;
    // 4: the tile's left column of x-faces (wave 0) and bottom row of
    // z-faces (wave 1), so that no wave runs both directions.
    const int kind2 = (z0 + r0 == nz - 1) ? FACE_TOP : FACE_INTERIOR;
    const int kind3 = (z0 + r0 + 1 == nz - 1) ? FACE_TOP : FACE_INTERIOR;
    // Edge faces: the x-face left of column 0 on each computed row, and the
    // z-face below the first computed row (tile row vs - 1 to vs).
    const bool ex_x4 = tid < TZ && tid >= vs && tid < ve;
    const int ez = tid - 64;
    const bool ex_z4 = ez >= 0 && ez < TX && ez < ncols;
    const int re = vs - 1;
    const int kind4 = (z0 + vs == 0) ? FACE_BOTTOM : FACE_INTERIOR;

    double F[5][NV];
    {
        const int cx[2] = {c, c}, rx[2] = {r0, r0 + 1};
        const int kx[2] = {FACE_INTERIOR, FACE_INTERIOR}, kz[2] = {kind2, kind3};
#if MPRK_FACE_PAIRS
        double Fp[2][NV];
        if (ok0 || ok1) {
            face_fluxes<DOM, 0, 2>(A, D, L, cx, rx, kx, Fp);
#pragma unroll
            for (int v = 0; v < NV; ++v) { F[0][v] = Fp[0][v]; F[1][v] = Fp[1][v]; }
            face_fluxes<DOM, 1, 2>(A, D, L, cx, rx, kz, Fp);
#pragma unroll
            for (int v = 0; v < NV; ++v) { F[2][v] = Fp[0][v]; F[3][v] = Fp[1][v]; }
        }
#else
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!(h ? ok1 : ok0)) continue;
            const int c1[1] = {c}, r1[1] = {rx[h]}, k1[1] = {FACE_INTERIOR}, k2[1] = {kz[h]};
            double Fs[1][NV];
            face_fluxes<DOM, 0, 1>(A, D, L, c1, r1, k1, Fs);
#pragma unroll
            for (int v = 0; v < NV; ++v) F[h][v] = Fs[0][v];
            FACE_SCHED_BARRIER();
            face_fluxes<DOM, 1, 1>(A, D, L, c1, r1, k2, Fs);
#pragma unroll
            for (int v = 0; v < NV; ++v) F[2 + h][v] = Fs[0][v];
            FACE_SCHED_BARRIER();
        }
#endif
        double Fs[1][NV];
        if (ex_x4) {
            const int c1[1] = {-1}, r1[1] = {tid}, k1[1] = {FACE_INTERIOR};
            face_fluxes<DOM, 0, 1>(A, D, L, c1, r1, k1, Fs);
#pragma unroll
            for (int v = 0; v < NV; ++v) F[4][v] = Fs[0][v];
        }
        if (ex_z4) {
            const int c1[1] = {ez}, r1[1] = {re}, k1[1] = {kind4};
            face_fluxes<DOM, 1, 1>(A, D, L, c1, r1, k1, Fs);
#pragma unroll
            for (int v = 0; v < NV; ++v) F[4][v] = Fs[0][v];
        }
    }

    // Pointwise global reads of the substep base U for the combination; they
    // complete while the fluxes are exchanged.
    const int col = x0 + c;
    const size_t plane = (size_t)nz * nx;
    const size_t nbx = (size_t)(D.b_hi - D.b_lo) * nx;
    double Ub[2][NV];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int row = z0 + r0 + h;
        const bool ok = h ? ok1 : ok0;
        const bool inb = (row >= D.b_lo && row < D.b_hi);
        const Combine& cb = inb ? D.buf : D.main;
        const size_t id = (size_t)row * nx + col;
#pragma unroll
        for (int v = 0; v < NV; ++v) Ub[h][v] = 0.0;
        if (ok && cb.mode != MODE_RHS && cb.alpha != 0.0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Ub[h][v] = D.base[v * plane + id];
        }
    }
    __syncthreads();   // all LDS reads of the staged state are done

    // Fluxes back from the face-normal frame to (rho, rho u, rho w, rho E).
    auto put_x = [&](int cc, int rr, const double* f) {
        double* e = ex_x + rr * (TX + 1) + cc + 1;
        constexpr int st = TZ * (TX + 1);
        e[0] = f[0]; e[st] = f[1]; e[2 * st] = f[2]; e[3 * st] = f[3];
    };
    auto put_z = [&](int cc, int rr, const double* f) {
        double* e = ex_z + (rr + 1) * TX + cc;
        constexpr int st = (TZ + 1) * TX;
        e[0] = f[0]; e[st] = f[2]; e[2 * st] = f[1]; e[3 * st] = f[3];
    };
    if (ok0) { put_x(c, r0, F[0]); put_z(c, r0, F[2]); }
    if (ok1) { put_x(c, r0 + 1, F[1]); put_z(c, r0 + 1, F[3]); }
    if (ex_x4) put_x(-1, tid, F[4]);
    if (ex_z4) put_z(ez, re, F[4]);
    __syncthreads();

    // ---- divergence, source and stage combination
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const bool ok = h ? ok1 : ok0;
        if (!ok) continue;
        const int r = r0 + h;
        const int row = z0 + r;
        double R[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double* fx = ex_x + v * TZ * (TX + 1) + r * (TX + 1) + c;
            const double* fz = ex_z + v * (TZ + 1) * TX + r * TX + c;
            R[v] = -(fx[1] - fx[0]) * A.inv_dx - (fz[TX] - fz[0]) * D.inv_dz;
        }
        R[2] += qc[h][0] * A.gravity;
        R[3] += qc[h][2] * A.gravity;

        const bool inb = (row >= D.b_lo && row < D.b_hi);
        const Combine& cb = inb ? D.buf : D.main;
        const size_t id = (size_t)row * nx + col;
        if (cb.mode == MODE_RHS) {
#pragma unroll
            for (int v = 0; v < NV; ++v) D.out[v * plane + id] = R[v];
        } else if (cb.alpha == 0.0) {
            // First stage of a base step: Qin is the base U itself.
#pragma unroll
            for (int v = 0; v < NV; ++v) D.out[v * plane + id] = qc[h][v] + cb.bh * R[v];
        } else {
            // Increment form of alpha U + beta (Qin + h R): U + beta (Qin - U)
            // + beta h R, exact when R = 0 and Qin = U.
            double inc[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) inc[v] = cb.beta * (qc[h][v] - Ub[h][v]) + cb.bh * R[v];
            if (cb.mode == MODE_STAGE) {
#pragma unroll
                for (int v = 0; v < NV; ++v) D.out[v * plane + id] = Ub[h][v] + inc[v];
            } else {
                // Buffer: accumulate the increments of the m trial steps and
                // add their mean to q^B_n after the last one.
                const size_t ia = (size_t)(row - D.b_lo) * nx + col;
                if (cb.mode == MODE_ACC_FIRST) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) D.acc[v * nbx + ia] = inc[v];
                } else if (cb.mode == MODE_ACC_ADD) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) D.acc[v * nbx + ia] += inc[v];
                } else {
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        D.out[v * plane + id] = Ub[h][v] + (D.acc[v * nbx + ia] + inc[v]) * A.inv_m;
                }
            }
        }
        if (D.ret_out && row >= D.ret_lo && row < D.ret_lo + 2) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                D.ret_out[(size_t)(v * 2 + row - D.ret_lo) * nx + col] = qc[h][v];
        }
    }
}

// Workgroups are dispatched to the 8 XCDs round-robin (block j to XCD j % 8).
// Give each XCD a contiguous range of the n tiles so that neighbouring tiles,
// which share halo rows and columns, meet in the same L2.
__device__ __forceinline__ int xcd_contiguous(int j, int n)
{
    constexpr int NXCD = 8;
    const int x = j % NXCD, i = j / NXCD;
    const int per = n / NXCD, rem = n % NXCD;
    return (x < rem) ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

#ifndef MPRK_WAVES_PER_EU
#define MPRK_WAVES_PER_EU 3
#endif

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MPRK_WAVES_PER_EU)))
void stage_kernel(const StageArgs A)
{
    __shared__ double lds[LDS_N];
    // Domain A.first takes the first blocks (the host puts the domain with
    // the shorter tiles first so they do not form a tail).
    const int b = blockIdx.x;
    const int n0 = A.d[A.first].ntiles;
    const int dom = (b < n0) ? A.first : 1 - A.first;
    int t = (b < n0) ? b : b - n0;
    // The second domain's blocks keep j % 8 == XCD only if n0 % 8 == 0.
    if (b < n0 || (n0 % 8) == 0) t = xcd_contiguous(t, (b < n0) ? n0 : A.nblocks - n0);
    if (dom == 0) stage_tile<0>(A, t, lds);
    else stage_tile<1>(A, t, lds);
}

// ---------------------------------------------------------------------------
// Persistent dataflow kernel.
// ---------------------------------------------------------------------------
// Wait until every tile this task reads has finished stage g - 1: the eight
// neighbours (x periodic) and, next to the interface, the tile across it.
// Called by the whole of wave 0: lane l < 9 polls neighbour (l%3 - 1, l/3 - 1),
// lane 9 the interface partner, all in parallel; a wave-wide vote decides.
// Returns false on timeout or abort; the kernel then exits without
// finishing (bounded: it never hangs).
__device__ bool wait_inputs(const PersistArgs& P, const MemberRun& M, const TileRef& tr, int g)
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
    const int64_t t0 = wall_clock64();
    while (true) {
        const bool ready = dep < 0 ||
            __hip_atomic_load(P.done + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        if (__all(ready)) break;
        __builtin_amdgcn_s_sleep(1);
        const bool ab = lane == 0 &&
            __hip_atomic_load(P.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        if (__any(ab) || wall_clock64() - t0 > P.wait_ticks) {
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

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MPRK_PERSIST_WAVES_PER_EU)))
void persistent_kernel(const PersistArgs P)
{
    __shared__ double lds[LDS_N];
    __shared__ int s_go;
    const int G = gridDim.x;
    for (int g = 1; g <= P.gmax; ++g) {
        // Blocks j and j + G run on the same XCD when G % 8 == 0; the remap
        // gives each XCD a contiguous range of tiles.
        for (int i = blockIdx.x; i < P.ntiles; i += G) {
            const int t = (G % 8 == 0) ? xcd_contiguous(i, P.ntiles) : i;
            const TileRef tr = P.tiles[t];
            const MemberRun& M = P.members[tr.member];
            if (g > M.nstages) continue;
            const StageArgs& A = M.stages[(g - 1) % M.ms];
            const DomainArgs& D = A.d[tr.dom];
            const int z0 = tr.tz * TZ;
            const bool work = D.row_hi > D.row_lo && z0 < D.row_hi && z0 + TZ > D.row_lo;
            if (work) {
                if (threadIdx.x < 64) {
                    const bool ok = wait_inputs(P, M, tr, g);
                    if (threadIdx.x == 0) s_go = ok ? 1 : 0;
                }
                __syncthreads();
                if (!s_go) return;
                const int rel = (tr.tz - D.row_lo / TZ) * D.tiles_x + tr.tx;
                if (tr.dom == 0) stage_tile<0>(A, rel, lds);
                else stage_tile<1>(A, rel, lds);
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
struct RedVal {
    double s[NV], e[NV];     // compensated sums: value + error term
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
    for (int v = 0; v < NV; ++v) {
        two_sum(a.s[v], a.e[v], b.s[v]);
        a.e[v] += b.e[v];
    }
    a.lam = fmax(a.lam, b.lam);
    a.cour = fmax(a.cour, b.cour);
    a.vis = fmax(a.vis, b.vis);
    a.bad = fmax(a.bad, b.bad);
}

__device__ __forceinline__ void red_store(double* p, const RedVal& a)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) { p[v] = a.s[v]; p[NV + v] = a.e[v]; }
    p[8] = a.lam; p[9] = a.cour; p[10] = a.vis; p[11] = a.bad;
}

__device__ __forceinline__ void red_load(const double* p, RedVal& a)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) { a.s[v] = p[v]; a.e[v] = p[NV + v]; }
    a.lam = p[8]; a.cour = p[9]; a.vis = p[10]; a.bad = p[11];
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

__global__ __launch_bounds__(RED_THREADS) void reduce_partial(const ReduceArgs A)
{
    __shared__ double sh[RED_THREADS * RED_FIELDS];
    const int dom = blockIdx.y;
    const double* q = A.q[dom];
    const int n = A.nz[dom] * A.nx;
    const double inv_dz = A.inv_dz[dom], vc = A.visc_coef[dom];
    RedVal m;
#pragma unroll
    for (int v = 0; v < NV; ++v) { m.s[v] = 0.0; m.e[v] = 0.0; }
    m.lam = m.cour = m.vis = m.bad = 0.0;
    for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) {
        const double rho = q[i], mx = q[(size_t)n + i], mz = q[2 * (size_t)n + i],
                     en = q[3 * (size_t)n + i];
        two_sum(m.s[0], m.e[0], rho);
        two_sum(m.s[1], m.e[1], mx);
        two_sum(m.s[2], m.e[2], mz);
        two_sum(m.s[3], m.e[3], en);
        const double ir = 1.0 / rho;
        const double u = mx * ir, w = mz * ir;
        const double p = A.gm1 * (en - 0.5 * (mx * u + mz * w));
        const bool ok = (rho > 0.0) && (p > 0.0) && isfinite(mx) && isfinite(mz) && isfinite(en);
        if (!ok) {
            m.bad = 1.0;
        } else {
            const double a = sqrt(A.gamma * p * ir);
            const double sx = (fabs(u) + a) * A.inv_dx;
            const double sz = (fabs(w) + a) * inv_dz;
            m.lam = fmax(m.lam, sx + sz);
            m.cour = fmax(m.cour, fmax(sx, sz));
            m.vis = fmax(m.vis, vc * ir);
        }
    }
    block_tree(m, sh);
    if (threadIdx.x == 0) red_store(A.partial + ((size_t)dom * RED_BLOCKS + blockIdx.x) * RED_FIELDS, m);
}

__global__ __launch_bounds__(RED_THREADS) void reduce_final(const ReduceArgs A)
{
    static_assert(RED_BLOCKS == RED_THREADS, "one partial per thread");
    __shared__ double sh[RED_THREADS * RED_FIELDS];
    const int dom = blockIdx.x;
    RedVal m;
    red_load(A.partial + ((size_t)dom * RED_BLOCKS + threadIdx.x) * RED_FIELDS, m);
    block_tree(m, sh);
    if (threadIdx.x == 0) red_store(A.final_ + (size_t)dom * RED_FIELDS, m);
}

}  // namespace

hipError_t launch_stage(const StageArgs& a, hipStream_t s)
{
    if (a.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(stage_kernel, dim3(a.nblocks), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_persistent(const PersistArgs& a, int grid, hipStream_t s)
{
    void* args[] = {(void*)&a};
    return hipLaunchCooperativeKernel((const void*)persistent_kernel, dim3(grid), dim3(NT), args, 0, s);
}

hipError_t launch_fill_i32(int32_t* p, int32_t value, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, value, n);
    return hipGetLastError();
}

int persistent_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)persistent_kernel, NT, 0) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_partial, dim3(RED_BLOCKS, 2), dim3(RED_THREADS), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final, dim3(2), dim3(RED_THREADS), 0, s, a);
    return hipGetLastError();
}

}  // namespace mprk
