/*
 * mprk_oracle3d.c -- FP64 CPU oracle of the three-dimensional coupled
 * two-domain compressible Navier-Stokes right-hand side (Appendix B,
 * eq. ns-fv-cartesian-3d) and its MPRK step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * HIP library.  Built together with mprk_oracle.c (whose MPRK tableaux it
 * uses), -O2 -ffp-contract=off, no fast-math.
 *
 * Plain on purpose: full temporary arrays, one face at a time, the Butcher
 * form with the expanded ms-stage tableaux.
 *
 * State: q[v][k][j][i], v = (rho, rho u, rho v, rho w, rho E), x fastest,
 * then y, then z (k = 0 the bottom plane).  x and y are periodic.
 *
 * Readings (in addition to those of the 2D file; listed in the design notes):
 *  - Mirror ghost plane (rho, rho u, rho v, -rho w, rho E) beyond walls and
 *    on each side of the interface.
 *  - Interface viscous flux in +z: (0, sigma_xz, sigma_yz, 0,
 *    u_w sigma_xz + v_w sigma_yz - Pi_z) with hat w = 0 and hat sigma_zz = 0
 *    (the rigid-lid simplification of Appendix B), u_w = u_1 +
 *    sigma_xz dz_1 / (2 mu_1), v_w = v_1 + sigma_yz dz_1 / (2 mu_1).
 *  - Viscous face fluxes: common velocity by averaging, normal derivatives by
 *    finite difference, tangential derivatives by averaging the two cells'
 *    central gradients (Appendix B); only the normal derivative of T enters
 *    (the heat flux through a face is -kappa dT/dn).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define N5 5
enum { R_ = 0, MU_ = 1, MV_ = 2, MW_ = 3, EN_ = 4 };

/* Shared with the Python wrapper (ctypes mirror). */
typedef struct {
    int32_t nx, ny;        /* cells in x and y (periodic), both domains      */
    int32_t nz_lower;      /* planes of the lower domain (Omega_1)           */
    int32_t nz_upper;      /* planes of the upper domain (Omega_2)           */
    int32_t fast_is_lower; /* 1: lower domain is the fast partition F        */
    int32_t n_buffer;      /* slow planes next to the interface forming B    */
    double dx, dy, dz_lower, dz_upper;
    double gamma, prandtl, mu_lower, mu_upper, gravity;
} orc3_cfg;

/* MPRK tableaux of the 2D file (same construction, dimension-free). */
int orc_tableau(int base, int m, double* aF, double* bF, double* cF, double* aB,
                double* bB, double* cB, double* aS, double* bS, double* cS);

/* Loops over fewer cells than this run on one thread (thread start-up would
 * cost more; results do not depend on the thread count). */
static inline int par3_ok(size_t cells) { return cells >= 16384; }

static inline size_t ix3(int nx, int ny, int nz, int v, int k, int j, int i)
{
    return (((size_t)v * (size_t)nz + (size_t)k) * (size_t)ny + (size_t)j) * (size_t)nx + (size_t)i;
}

static inline int per(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* ---- physics (Section 2, eq. cns-gov; EOS p = rho T / gamma) ------------ */
static double pres3(const double q[N5], double gamma)
{
    double u = q[MU_] / q[R_], v = q[MV_] / q[R_], w = q[MW_] / q[R_];
    return (gamma - 1.0) * (q[EN_] - 0.5 * q[R_] * (u * u + v * v + w * w));
}

/* Physical inviscid flux in direction d (0 x, 1 y, 2 z): F, G or H of
 * Appendix B. */
static void flux3(const double q[N5], int d, double gamma, double f[N5])
{
    double p = pres3(q, gamma);
    double un = q[MU_ + d] / q[R_];
    f[R_] = q[R_] * un;
    f[MU_] = q[MU_] * un + (d == 0 ? p : 0.0);
    f[MV_] = q[MV_] * un + (d == 1 ? p : 0.0);
    f[MW_] = q[MW_] * un + (d == 2 ? p : 0.0);
    f[EN_] = (q[EN_] + p) * un;
}

/* Local Lax-Friedrichs flux with lambda = max |u_n| + a over the two states
 * and their Roe average. */
static void llf3(const double qL[N5], const double qR[N5], int d, double gamma, double F[N5])
{
    double fL[N5], fR[N5];
    flux3(qL, d, gamma, fL);
    flux3(qR, d, gamma, fR);
    double uL[3], uR[3];
    for (int c = 0; c < 3; ++c) {
        uL[c] = qL[MU_ + c] / qL[R_];
        uR[c] = qR[MU_ + c] / qR[R_];
    }
    double pL = pres3(qL, gamma), pR = pres3(qR, gamma);
    double aL = sqrt(gamma * pL / qL[R_]), aR = sqrt(gamma * pR / qR[R_]);
    double HL = (qL[EN_] + pL) / qL[R_], HR = (qR[EN_] + pR) / qR[R_];
    double sL = sqrt(qL[R_]), sR = sqrt(qR[R_]);
    double ur[3];
    for (int c = 0; c < 3; ++c) ur[c] = (sL * uL[c] + sR * uR[c]) / (sL + sR);
    double Hr = (sL * HL + sR * HR) / (sL + sR);
    double ar = sqrt((gamma - 1.0) * (Hr - 0.5 * (ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2])));
    double lam = fabs(uL[d]) + aL;
    if (fabs(uR[d]) + aR > lam) lam = fabs(uR[d]) + aR;
    if (fabs(ur[d]) + ar > lam) lam = fabs(ur[d]) + ar;
    for (int v = 0; v < N5; ++v) F[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * (qR[v] - qL[v]);
}

static void mirror3(const double q[N5], double m[N5])
{
    memcpy(m, q, sizeof(double) * N5);
    m[MW_] = -q[MW_];
}

static double kappa3(double mu, double gamma, double prandtl)
{
    return mu / ((gamma - 1.0) * prandtl);
}

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz, mu, kappa, gamma, gravity;
} dom3_t;

/*
 * One domain's RHS on planes [k_lo, k_hi).  bot_gamma / top_gamma select the
 * lid below / above (else a slip adiabatic wall); fvg is the per-column
 * (j, i) interface viscous flux in +z, N5 components.
 */
static void domain_rhs3(const dom3_t* D, const double* q, const double* fvg, int bot_gamma,
                        int top_gamma, double* r, int k_lo, int k_hi)
{
    const int nx = D->nx, ny = D->ny, nz = D->nz, ne = nz + 2;
    const size_t pl = (size_t)nx * ny;
    const double gm = D->gamma;
    if (k_lo < 0) k_lo = 0;
    if (k_hi > nz) k_hi = nz;
    if (k_lo >= k_hi) return;

    double* qe = (double*)malloc(sizeof(double) * N5 * ne * pl);   /* with ghost planes */
    double* pe = (double*)malloc(sizeof(double) * 4 * ne * pl);    /* u, v, w, T */
    double* dq = (double*)malloc(sizeof(double) * 3 * N5 * nz * pl);  /* d/dx, d/dy, d/dz */
    double* du = (double*)malloc(sizeof(double) * 9 * nz * pl);    /* [c*3+d]: d u_c / d x_d */
    double* Fx = (double*)malloc(sizeof(double) * N5 * nz * pl);   /* face i+1/2 */
    double* Fy = (double*)malloc(sizeof(double) * N5 * nz * pl);   /* face j+1/2 */
    double* Fz = (double*)malloc(sizeof(double) * N5 * (nz + 1) * pl);  /* below plane f */
#define QE(v, e, j, i) qe[ix3(nx, ny, ne, v, e, j, i)]
#define PE(f, e, j, i) pe[ix3(nx, ny, ne, f, e, j, i)]
#define DQ(d, v, k, j, i) dq[ix3(nx, ny, nz, (d) * N5 + (v), k, j, i)]
#define DU(c, d, k, j, i) du[ix3(nx, ny, nz, (c) * 3 + (d), k, j, i)]

#pragma omp parallel for schedule(static) if (par3_ok(pl * (size_t)nz))
    for (int e = 0; e < ne; ++e) {
        int k = e - 1;
        int src = k < 0 ? 0 : (k >= nz ? nz - 1 : k);
        int ghost = (k < 0 || k >= nz);
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double c[N5], g[N5];
                for (int v = 0; v < N5; ++v) c[v] = q[ix3(nx, ny, nz, v, src, j, i)];
                if (ghost) mirror3(c, g); else memcpy(g, c, sizeof g);
                for (int v = 0; v < N5; ++v) QE(v, e, j, i) = g[v];
                for (int cc = 0; cc < 3; ++cc) PE(cc, e, j, i) = g[MU_ + cc] / g[R_];
                PE(3, e, j, i) = gm * pres3(g, gm) / g[R_];
            }
    }

    /* Cell gradients by central differences (the least-squares gradient on a
     * uniform grid, Appendix B footnote), using the ghost planes. */
#pragma omp parallel for schedule(static) if (par3_ok(pl * (size_t)nz))
    for (int k = 0; k < nz; ++k) {
        int e = k + 1;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int im = per(i - 1, nx), ip = per(i + 1, nx);
                int jm = per(j - 1, ny), jp = per(j + 1, ny);
                for (int v = 0; v < N5; ++v) {
                    DQ(0, v, k, j, i) = (QE(v, e, j, ip) - QE(v, e, j, im)) / (2.0 * D->dx);
                    DQ(1, v, k, j, i) = (QE(v, e, jp, i) - QE(v, e, jm, i)) / (2.0 * D->dy);
                    DQ(2, v, k, j, i) = (QE(v, e + 1, j, i) - QE(v, e - 1, j, i)) / (2.0 * D->dz);
                }
                for (int c = 0; c < 3; ++c) {
                    DU(c, 0, k, j, i) = (PE(c, e, j, ip) - PE(c, e, j, im)) / (2.0 * D->dx);
                    DU(c, 1, k, j, i) = (PE(c, e, jp, i) - PE(c, e, jm, i)) / (2.0 * D->dy);
                    DU(c, 2, k, j, i) = (PE(c, e + 1, j, i) - PE(c, e - 1, j, i)) / (2.0 * D->dz);
                }
            }
    }

    /* x- and y-faces on the requested planes. */
#pragma omp parallel for schedule(static) if (par3_ok(pl * (size_t)nz))
    for (int k = k_lo; k < k_hi; ++k) {
        int e = k + 1;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                for (int d = 0; d < 2; ++d) {
                    int i2 = d == 0 ? per(i + 1, nx) : i;
                    int j2 = d == 1 ? per(j + 1, ny) : j;
                    double h = d == 0 ? D->dx : D->dy;
                    double qL[N5], qR[N5], F[N5];
                    for (int v = 0; v < N5; ++v) {
                        qL[v] = QE(v, e, j, i) + DQ(d, v, k, j, i) * (h / 2.0);
                        qR[v] = QE(v, e, j2, i2) - DQ(d, v, k, j2, i2) * (h / 2.0);
                    }
                    llf3(qL, qR, d, gm, F);
                    double uh[3], g[3][3];     /* common velocity and gradient g[c][dir] */
                    for (int c = 0; c < 3; ++c) {
                        uh[c] = 0.5 * (PE(c, e, j, i) + PE(c, e, j2, i2));
                        for (int t = 0; t < 3; ++t)
                            g[c][t] = (t == d) ? (PE(c, e, j2, i2) - PE(c, e, j, i)) / h
                                               : 0.5 * (DU(c, t, k, j, i) + DU(c, t, k, j2, i2));
                    }
                    double Tn = (PE(3, e, j2, i2) - PE(3, e, j, i)) / h;
                    /* sigma = mu (grad u + grad u^T - 2/3 I div u), Section 2:
                     * sigma_dd = mu (4/3 g_dd - 2/3 (sum of the other two)). */
                    double s[3];               /* sigma_{d c}, c = x, y, z */
                    for (int c = 0; c < 3; ++c)
                        s[c] = (c == d) ? D->mu * (4.0 / 3.0 * g[d][d] -
                                                   2.0 / 3.0 * (g[(d + 1) % 3][(d + 1) % 3] +
                                                                g[(d + 2) % 3][(d + 2) % 3]))
                                        : D->mu * (g[d][c] + g[c][d]);
                    double fv[N5] = {0.0, s[0], s[1], s[2],
                                     uh[0] * s[0] + uh[1] * s[1] + uh[2] * s[2] + D->kappa * Tn};
                    double* out = d == 0 ? Fx : Fy;
                    for (int v = 0; v < N5; ++v) out[ix3(nx, ny, nz, v, k, j, i)] = F[v] - fv[v];
                }
            }
    }

    /* z-faces f = k_lo .. k_hi (below plane f). */
#pragma omp parallel for schedule(static) if (par3_ok(pl * (size_t)nz))
    for (int f = k_lo; f <= k_hi; ++f) {
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double qL[N5], qR[N5], F[N5], fv[N5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                if (f == 0 || f == nz) {
                    int k = (f == 0) ? 0 : nz - 1;
                    double sgn = (f == 0) ? -1.0 : 1.0, qh[N5];
                    for (int v = 0; v < N5; ++v)
                        qh[v] = q[ix3(nx, ny, nz, v, k, j, i)] + sgn * DQ(2, v, k, j, i) * (D->dz / 2.0);
                    if (f == 0) { mirror3(qh, qL); memcpy(qR, qh, sizeof qR); }
                    else        { memcpy(qL, qh, sizeof qL); mirror3(qh, qR); }
                    llf3(qL, qR, 2, gm, F);
                    int is_gamma = (f == 0) ? bot_gamma : top_gamma;
                    if (is_gamma)
                        for (int v = 0; v < N5; ++v) fv[v] = fvg[((size_t)j * nx + i) * N5 + v];
                } else {
                    int kl = f - 1, kr = f;
                    for (int v = 0; v < N5; ++v) {
                        qL[v] = q[ix3(nx, ny, nz, v, kl, j, i)] + DQ(2, v, kl, j, i) * (D->dz / 2.0);
                        qR[v] = q[ix3(nx, ny, nz, v, kr, j, i)] - DQ(2, v, kr, j, i) * (D->dz / 2.0);
                    }
                    llf3(qL, qR, 2, gm, F);
                    int eL = kl + 1, eR = kr + 1;
                    double uh[3], g[3][3];
                    for (int c = 0; c < 3; ++c) {
                        uh[c] = 0.5 * (PE(c, eL, j, i) + PE(c, eR, j, i));
                        for (int t = 0; t < 3; ++t)
                            g[c][t] = (t == 2) ? (PE(c, eR, j, i) - PE(c, eL, j, i)) / D->dz
                                               : 0.5 * (DU(c, t, kl, j, i) + DU(c, t, kr, j, i));
                    }
                    double Tn = (PE(3, eR, j, i) - PE(3, eL, j, i)) / D->dz;
                    double s[3];
                    for (int c = 0; c < 3; ++c)
                        s[c] = (c == 2) ? D->mu * (4.0 / 3.0 * g[2][2] - 2.0 / 3.0 * (g[0][0] + g[1][1]))
                                        : D->mu * (g[2][c] + g[c][2]);
                    fv[1] = s[0];
                    fv[2] = s[1];
                    fv[3] = s[2];
                    fv[4] = uh[0] * s[0] + uh[1] * s[1] + uh[2] * s[2] + D->kappa * Tn;
                }
                for (int v = 0; v < N5; ++v) Fz[ix3(nx, ny, nz + 1, v, f, j, i)] = F[v] - fv[v];
            }
    }

    /* Divergence plus source (0, 0, 0, rho g, rho w g). */
#pragma omp parallel for schedule(static) if (par3_ok(pl * (size_t)nz))
    for (int k = k_lo; k < k_hi; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int im = per(i - 1, nx), jm = per(j - 1, ny);
                double rho = q[ix3(nx, ny, nz, R_, k, j, i)];
                double mw = q[ix3(nx, ny, nz, MW_, k, j, i)];
                double src[N5] = {0.0, 0.0, 0.0, rho * D->gravity, mw * D->gravity};
                for (int v = 0; v < N5; ++v) {
                    double dfx = (Fx[ix3(nx, ny, nz, v, k, j, i)] - Fx[ix3(nx, ny, nz, v, k, j, im)]) / D->dx;
                    double dfy = (Fy[ix3(nx, ny, nz, v, k, j, i)] - Fy[ix3(nx, ny, nz, v, k, jm, i)]) / D->dy;
                    double dfz = (Fz[ix3(nx, ny, nz + 1, v, k + 1, j, i)] -
                                  Fz[ix3(nx, ny, nz + 1, v, k, j, i)]) / D->dz;
                    r[ix3(nx, ny, nz, v, k, j, i)] = -dfx - dfy - dfz + src[v];
                }
            }
#undef QE
#undef PE
#undef DQ
#undef DU
    free(qe); free(pe); free(dq); free(du); free(Fx); free(Fy); free(Fz);
}

/* Interface quantities per column from the two cells next to Gamma (index 1
 * lower, 2 upper): out[c*8 + {0..7}] = sigma_xz, sigma_yz, Pi_z, u_w1, v_w1,
 * T_w1, u_w2, v_w2. */
static void interface3(const orc3_cfg* c, const double* qlo, const double* qup, double* out)
{
    const int nx = c->nx, ny = c->ny;
    double k1 = kappa3(c->mu_lower, c->gamma, c->prandtl);
    double k2 = kappa3(c->mu_upper, c->gamma, c->prandtl);
    double mu1 = c->mu_lower, mu2 = c->mu_upper, dz1 = c->dz_lower, dz2 = c->dz_upper;
    double bu = 2.0 * mu1 * mu2 / (dz2 * mu1 + dz1 * mu2);
    double bT = 2.0 * k1 * k2 / (dz2 * k1 + dz1 * k2);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double a[N5], b[N5];
            for (int v = 0; v < N5; ++v) {
                a[v] = qlo[ix3(nx, ny, c->nz_lower, v, c->nz_lower - 1, j, i)];
                b[v] = qup[ix3(nx, ny, c->nz_upper, v, 0, j, i)];
            }
            double u1 = a[MU_] / a[R_], v1 = a[MV_] / a[R_], T1 = c->gamma * pres3(a, c->gamma) / a[R_];
            double u2 = b[MU_] / b[R_], v2 = b[MV_] / b[R_], T2 = c->gamma * pres3(b, c->gamma) / b[R_];
            double sxz = bu * (u2 - u1), syz = bu * (v2 - v1), piz = -bT * (T2 - T1);
            double* o = out + ((size_t)j * nx + i) * 8;
            o[0] = sxz;
            o[1] = syz;
            o[2] = piz;
            o[3] = u1 + sxz * dz1 / (2.0 * mu1);
            o[4] = v1 + syz * dz1 / (2.0 * mu1);
            o[5] = T1 - piz * dz1 / (2.0 * k1);
            o[6] = u2 - sxz * dz2 / (2.0 * mu2);
            o[7] = v2 - syz * dz2 / (2.0 * mu2);
        }
}

static void coupled_rhs3(const orc3_cfg* c, const double* qlo, const double* qup, double* rlo,
                         double* rup, int lo0, int hi0, int lo1, int hi1)
{
    const size_t pl = (size_t)c->nx * c->ny;
    double* ifc = (double*)malloc(sizeof(double) * 8 * pl);
    double* fvg = (double*)malloc(sizeof(double) * N5 * pl);
    interface3(c, qlo, qup, ifc);
    for (size_t p = 0; p < pl; ++p) {
        const double* o = ifc + p * 8;
        fvg[p * N5 + 0] = 0.0;
        fvg[p * N5 + 1] = o[0];
        fvg[p * N5 + 2] = o[1];
        fvg[p * N5 + 3] = 0.0;
        fvg[p * N5 + 4] = o[3] * o[0] + o[4] * o[1] - o[2];
    }
    dom3_t L = {c->nx, c->ny, c->nz_lower, c->dx, c->dy, c->dz_lower, c->mu_lower,
                kappa3(c->mu_lower, c->gamma, c->prandtl), c->gamma, c->gravity};
    dom3_t U = {c->nx, c->ny, c->nz_upper, c->dx, c->dy, c->dz_upper, c->mu_upper,
                kappa3(c->mu_upper, c->gamma, c->prandtl), c->gamma, c->gravity};
    domain_rhs3(&L, qlo, fvg, 0, 1, rlo, lo0, hi0);
    domain_rhs3(&U, qup, fvg, 1, 0, rup, lo1, hi1);
    free(ifc);
    free(fvg);
}

int orc3_rhs(const orc3_cfg* c, const double* qlo, const double* qup, double* rlo, double* rup)
{
    coupled_rhs3(c, qlo, qup, rlo, rup, 0, c->nz_lower, 0, c->nz_upper);
    return 0;
}

int orc3_interface(const orc3_cfg* c, const double* qlo, const double* qup, double* out)
{
    interface3(c, qlo, qup, out);
    return 0;
}

int orc3_llf(const double* qL, const double* qR, int d, double gamma, double* F)
{
    llf3(qL, qR, d, gamma, F);
    return 0;
}

/* One MPRK step in Butcher form (Algorithm 1; the same schedule as the 2D
 * oracle's step, over planes instead of rows). */
int orc3_mprk_step(const orc3_cfg* c, int base, int m, double dt, double* qlo, double* qup)
{
    if (base != 2 && base != 3) return -1;
    if (m < 1) return -1;
    const int s = base, ms = m * s;
    double* aF = (double*)malloc(sizeof(double) * ms * ms);
    double* aB = (double*)malloc(sizeof(double) * ms * ms);
    double* aS = (double*)malloc(sizeof(double) * ms * ms);
    double* bF = (double*)malloc(sizeof(double) * ms);
    double* bB = (double*)malloc(sizeof(double) * ms);
    double* bS = (double*)malloc(sizeof(double) * ms);
    double* cF = (double*)malloc(sizeof(double) * ms);
    double* cB = (double*)malloc(sizeof(double) * ms);
    double* cS = (double*)malloc(sizeof(double) * ms);
    orc_tableau(base, m, aF, bF, cF, aB, bB, cB, aS, bS, cS);

    const size_t pl = (size_t)c->nx * c->ny;
    double* qF = c->fast_is_lower ? qlo : qup;
    double* qSl = c->fast_is_lower ? qup : qlo;
    const int nzF = c->fast_is_lower ? c->nz_lower : c->nz_upper;
    const int nzS = c->fast_is_lower ? c->nz_upper : c->nz_lower;
    int b_lo, b_hi;
    if (c->fast_is_lower) { b_lo = 0; b_hi = c->n_buffer; }
    else { b_lo = c->nz_lower - c->n_buffer; b_hi = c->nz_lower; }
    const size_t nF = (size_t)N5 * nzF * pl, nS = (size_t)N5 * nzS * pl;
    double* RF = (double*)calloc((size_t)ms * nF, sizeof(double));
    double* RS = (double*)calloc((size_t)ms * nS, sizeof(double));
    double* QF = (double*)malloc(sizeof(double) * nF);
    double* QS = (double*)malloc(sizeof(double) * nS);
    double* Ssave = (double*)malloc(sizeof(double) * (size_t)s * nS);

    for (int i = 0; i < ms; ++i) {
#pragma omp parallel for schedule(static) if (par3_ok(pl * (size_t)(nzF + nzS)))
        for (int k = 0; k < nzS; ++k) {
            int in_b = (k >= b_lo && k < b_hi);
            for (int v = 0; v < N5; ++v)
                for (size_t p = 0; p < pl; ++p) {
                    size_t id = ((size_t)v * nzS + k) * pl + p;
                    if (in_b) {
                        double acc = 0.0;
                        for (int j = 0; j < i; ++j) acc += aB[i * ms + j] * RS[(size_t)j * nS + id];
                        QS[id] = qSl[id] + dt * acc;
                    } else if (i < s) {
                        double acc = 0.0;
                        for (int j = 0; j < i; ++j) acc += aS[i * ms + j] * RS[(size_t)j * nS + id];
                        QS[id] = qSl[id] + dt * acc;
                        Ssave[(size_t)i * nS + id] = QS[id];
                    } else {
                        QS[id] = Ssave[(size_t)(i % s) * nS + id];   /* copy line */
                    }
                }
        }
#pragma omp parallel for schedule(static) if (par3_ok(pl * (size_t)(nzF + nzS)))
        for (int k = 0; k < nzF; ++k)
            for (int v = 0; v < N5; ++v)
                for (size_t p = 0; p < pl; ++p) {
                    size_t id = ((size_t)v * nzF + k) * pl + p;
                    double acc = 0.0;
                    for (int j = 0; j < i; ++j) acc += aF[i * ms + j] * RF[(size_t)j * nF + id];
                    QF[id] = qF[id] + dt * acc;
                }
        int s_lo = (i < s) ? 0 : b_lo, s_hi = (i < s) ? nzS : b_hi;
        double* rF = RF + (size_t)i * nF;
        double* rS = RS + (size_t)i * nS;
        if (c->fast_is_lower) coupled_rhs3(c, QF, QS, rF, rS, 0, nzF, s_lo, s_hi);
        else coupled_rhs3(c, QS, QF, rS, rF, s_lo, s_hi, 0, nzF);
    }
#pragma omp parallel for schedule(static) if (par3_ok(pl * (size_t)(nzF + nzS)))
    for (int k = 0; k < nzF; ++k)
        for (int v = 0; v < N5; ++v)
            for (size_t p = 0; p < pl; ++p) {
                size_t id = ((size_t)v * nzF + k) * pl + p;
                double acc = 0.0;
                for (int i = 0; i < ms; ++i) acc += bF[i] * RF[(size_t)i * nF + id];
                qF[id] = qF[id] + dt * acc;
            }
#pragma omp parallel for schedule(static) if (par3_ok(pl * (size_t)(nzF + nzS)))
    for (int k = 0; k < nzS; ++k) {
        int in_b = (k >= b_lo && k < b_hi);
        for (int v = 0; v < N5; ++v)
            for (size_t p = 0; p < pl; ++p) {
                size_t id = ((size_t)v * nzS + k) * pl + p;
                double acc = 0.0;
                if (in_b) for (int i = 0; i < ms; ++i) acc += bB[i] * RS[(size_t)i * nS + id];
                else for (int i = 0; i < s; ++i) acc += bS[i] * RS[(size_t)i * nS + id];
                qSl[id] = qSl[id] + dt * acc;
            }
    }
    free(aF); free(aB); free(aS); free(bF); free(bB); free(bS); free(cF); free(cB); free(cS);
    free(RF); free(RS); free(QF); free(QS); free(Ssave);
    return 0;
}

int orc3_mprk_run(const orc3_cfg* c, int base, int m, double dt, int64_t n, double* qlo, double* qup)
{
    for (int64_t t = 0; t < n; ++t) {
        int rc = orc3_mprk_step(c, base, m, dt, qlo, qup);
        if (rc) return rc;
    }
    return 0;
}

/* Neumaier-compensated totals: out[0..4] lower, out[5..9] upper. */
int orc3_totals(const orc3_cfg* c, const double* qlo, const double* qup, double* out)
{
    const size_t pl = (size_t)c->nx * c->ny;
    for (int d = 0; d < 2; ++d) {
        const double* q = d == 0 ? qlo : qup;
        int nz = d == 0 ? c->nz_lower : c->nz_upper;
        double vol = c->dx * c->dy * (d == 0 ? c->dz_lower : c->dz_upper);
        for (int v = 0; v < N5; ++v) {
            double s = 0.0, comp = 0.0;
            for (size_t id = 0; id < (size_t)nz * pl; ++id) {
                double x = q[(size_t)v * nz * pl + id];
                double t = s + x;
                if (fabs(s) >= fabs(x)) comp += (s - t) + x;
                else comp += (x - t) + s;
                s = t;
            }
            out[d * N5 + v] = (s + comp) * vol;
        }
    }
    return 0;
}

/* Stability measures per domain (as the 2D file, with the y direction):
 * lam = max sum_d (|u_d| + a)/h_d, cour = max over cells and directions,
 * vis = max max(4/3, gamma/Pr) mu / rho sum_d 1/h_d^2.  Returns 1 on a bad
 * state. */
int orc3_wave_measures(const orc3_cfg* c, const double* qlo, const double* qup, double* lam,
                       double* cour, double* vis)
{
    int bad = 0;
    const size_t pl = (size_t)c->nx * c->ny;
    double coef = 4.0 / 3.0;
    if (c->gamma / c->prandtl > coef) coef = c->gamma / c->prandtl;
    for (int d = 0; d < 2; ++d) {
        const double* q = d == 0 ? qlo : qup;
        int nz = d == 0 ? c->nz_lower : c->nz_upper;
        double h[3] = {c->dx, c->dy, d == 0 ? c->dz_lower : c->dz_upper};
        double mu = d == 0 ? c->mu_lower : c->mu_upper;
        double L = 0.0, C = 0.0, V = 0.0;
        for (size_t id = 0; id < (size_t)nz * pl; ++id) {
            double cc[N5];
            for (int v = 0; v < N5; ++v) cc[v] = q[(size_t)v * nz * pl + id];
            double p = pres3(cc, c->gamma);
            int ok = cc[R_] > 0.0 && p > 0.0;
            for (int v = 0; v < N5; ++v) ok = ok && isfinite(cc[v]);
            if (!ok) { bad = 1; continue; }
            double a = sqrt(c->gamma * p / cc[R_]);
            double sum = 0.0, inv2 = 0.0;
            for (int t = 0; t < 3; ++t) {
                double sd = (fabs(cc[MU_ + t] / cc[R_]) + a) / h[t];
                sum += sd;
                if (sd > C) C = sd;
                inv2 += 1.0 / (h[t] * h[t]);
            }
            if (sum > L) L = sum;
            double vv = coef * mu / cc[R_] * inv2;
            if (vv > V) V = vv;
        }
        lam[d] = L;
        cour[d] = C;
        vis[d] = V;
    }
    return bad;
}

double orc3_dt_rule(const orc3_cfg* c, const double* qlo, const double* qup, int m, double cr,
                    double dn)
{
    double lam[2], cour[2], vis[2];
    if (orc3_wave_measures(c, qlo, qup, lam, cour, vis)) return 0.0;
    int f = c->fast_is_lower ? 0 : 1, sl = 1 - f;
    double dtf = 1.0 / (lam[f] / cr + vis[f] / dn);
    double dts = 1.0 / (lam[sl] / cr + vis[sl] / dn);
    double dt = m * dtf;
    if (dts < dt) dt = dts;
    return dt;
}
