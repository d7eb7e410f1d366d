/*
 * mprk_oracle.c -- FP64 CPU oracle for the coupled two-domain compressible
 * Navier-Stokes (CNS) right-hand side and the multirate partitioned
 * Runge-Kutta (MPRK) step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * It is deliberately plain: nested loops, one face at a time, full temporary
 * arrays, Butcher form with the expanded ms-stage tableaux.  It is built with
 * -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 *
 * Paper: Kang, Dener, Hamilton, Zhang, Constantinescu, Jacob, "Multirate
 * partitioned Runge-Kutta methods for coupled Navier-Stokes equations"
 * (arXiv 2202.11890).  Citations below name the paper's section, equation,
 * table or algorithm.
 *
 * Readings where the paper is silent or garbled (each is listed in the design
 * notes of the repository):
 *  - 2D model = Appendix B restricted to the x-z plane, q = (rho, rho u,
 *    rho w, rho E).
 *  - Inviscid flux: scalar local Lax-Friedrichs, 1/2 (f(qL)+f(qR)).n
 *    - 1/2 lambda (qR - qL); lambda = max of |u_n|+a over qL, qR and their
 *    Roe average (sqrt(rho)-weighted velocity and total enthalpy).
 *  - Reconstruction of conserved variables, no limiter.
 *  - Mirror ghost row (rho, rho u, -rho w, rho E) beyond walls and on each
 *    side of the interface, for all cell gradients.
 *  - Slip adiabatic walls: LLF of the reconstructed wall state and its mirror,
 *    zero viscous flux.
 *  - Heat flux Pi = -kappa grad T with kappa = mu / ((gamma-1) Pr).
 *  - Interface viscous flux (0, sigma_xz, 0, u_w sigma_xz - Pi_z), computed
 *    once per column and used by both domains; each domain keeps its own
 *    reflective inviscid flux there.
 *  - Source (0, 0, rho g, rho w g) with g the signed vertical gravity.
 *  - MPRK tableaux for any (m, s) built from the base tableau as described in
 *    orc_tableau(); they reproduce Table 1 for m = s = 2.
 *
 * Pins: every function here is checked against values fixed by the paper or
 * by mathematics (tests/test_oracle_*.py).  orc_mprk_step's multirate
 * partition logic is pinned by conservation, by m = 1 reducing to the
 * separately coded single-rate loop, and by the temporal order; no printed
 * trajectory exists to compare with.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 4
enum { I_RHO = 0, I_MX = 1, I_MZ = 2, I_EN = 3 };

/* Problem description shared with the Python wrapper (ctypes mirror). */
typedef struct {
    int32_t nx;            /* cells in x (periodic), both domains            */
    int32_t nz_lower;      /* rows of the lower domain (Omega_1)             */
    int32_t nz_upper;      /* rows of the upper domain (Omega_2)             */
    int32_t fast_is_lower; /* 1: lower domain is the fast partition F        */
    int32_t n_buffer;      /* slow rows next to the interface forming B      */
    int32_t pad;
    double dx, dz_lower, dz_upper;
    double gamma, prandtl, mu_lower, mu_upper, gravity;
} orc_cfg;

/* ------------------------------------------------------------------------ */
/* Indexing: q[v][k][i], x fastest, k = 0 is the bottom row.                */
/* ------------------------------------------------------------------------ */
/* Loops over fewer cells than this run on one thread: thread start-up would
 * cost more than the loop (results do not depend on the thread count, every
 * output element being written by exactly one iteration). */
#define ORC_PAR_MIN_CELLS 16384
static inline int par_ok(size_t cells) { return cells >= ORC_PAR_MIN_CELLS; }

static inline size_t at(int nx, int nz, int v, int k, int i)
{
    return ((size_t)v * (size_t)nz + (size_t)k) * (size_t)nx + (size_t)i;
}

static inline int wrap(int i, int nx)
{
    int r = i % nx;
    return r < 0 ? r + nx : r;
}

/* ------------------------------------------------------------------------ */
/* Physics (Section 2, eq. cns-gov; Appendix A, nondimensional EOS          */
/* p = rho T / gamma, so the sound speed is a = sqrt(gamma p / rho).)       */
/* ------------------------------------------------------------------------ */
static double pressure(const double q[NV], double gamma)
{
    double u = q[I_MX] / q[I_RHO];
    double w = q[I_MZ] / q[I_RHO];
    return (gamma - 1.0) * (q[I_EN] - 0.5 * q[I_RHO] * (u * u + w * w));
}

/* Physical inviscid flux in direction dir (0: x, 1: z): (rho u_n,
 * rho u u_n + p n, rho H u_n) with rho H = rho E + p. */
static void inviscid_flux(const double q[NV], int dir, double gamma, double f[NV])
{
    double u = q[I_MX] / q[I_RHO];
    double w = q[I_MZ] / q[I_RHO];
    double p = pressure(q, gamma);
    double un = dir == 0 ? u : w;
    f[I_RHO] = q[I_RHO] * un;
    f[I_MX] = q[I_MX] * un + (dir == 0 ? p : 0.0);
    f[I_MZ] = q[I_MZ] * un + (dir == 1 ? p : 0.0);
    f[I_EN] = (q[I_EN] + p) * un;
}

/* Local Lax-Friedrichs flux (Section 2.1, numerical flux; lambda from the
 * left, right and Roe-average states). */
static void llf_flux(const double qL[NV], const double qR[NV], int dir,
                     double gamma, double F[NV])
{
    double fL[NV], fR[NV];
    inviscid_flux(qL, dir, gamma, fL);
    inviscid_flux(qR, dir, gamma, fR);

    double uL = qL[I_MX] / qL[I_RHO], wL = qL[I_MZ] / qL[I_RHO];
    double uR = qR[I_MX] / qR[I_RHO], wR = qR[I_MZ] / qR[I_RHO];
    double pL = pressure(qL, gamma), pR = pressure(qR, gamma);
    double aL = sqrt(gamma * pL / qL[I_RHO]);
    double aR = sqrt(gamma * pR / qR[I_RHO]);
    double HL = (qL[I_EN] + pL) / qL[I_RHO];
    double HR = (qR[I_EN] + pR) / qR[I_RHO];
    double unL = dir == 0 ? uL : wL;
    double unR = dir == 0 ? uR : wR;

    /* Roe average: weights sqrt(rho). */
    double sL = sqrt(qL[I_RHO]), sR = sqrt(qR[I_RHO]);
    double ur = (sL * uL + sR * uR) / (sL + sR);
    double wr = (sL * wL + sR * wR) / (sL + sR);
    double Hr = (sL * HL + sR * HR) / (sL + sR);
    double ar = sqrt((gamma - 1.0) * (Hr - 0.5 * (ur * ur + wr * wr)));
    double unr = dir == 0 ? ur : wr;

    double lam = fabs(unL) + aL;
    if (fabs(unR) + aR > lam) lam = fabs(unR) + aR;
    if (fabs(unr) + ar > lam) lam = fabs(unr) + ar;

    for (int v = 0; v < NV; ++v)
        F[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * (qR[v] - qL[v]);
}

/* Mirror state across a horizontal wall or the rigid lid. */
static void mirror(const double q[NV], double m[NV])
{
    m[I_RHO] = q[I_RHO];
    m[I_MX] = q[I_MX];
    m[I_MZ] = -q[I_MZ];
    m[I_EN] = q[I_EN];
}

/* ------------------------------------------------------------------------ */
/* Interface (rigid lid) coupling, Appendix B eq. (bulk-flux) and the wall  */
/* state formulas that follow it.  Index 1 = lower cell next to Gamma,      */
/* index 2 = upper cell next to Gamma.                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double sigma_xz, pi_z, uw1, uw2, tw1, tw2;
} iface_t;

static iface_t interface_column(double u1, double T1, double u2, double T2,
                                double mu1, double mu2, double kap1, double kap2,
                                double dz1, double dz2)
{
    iface_t r;
    double bu = 2.0 * mu1 * mu2 / (dz2 * mu1 + dz1 * mu2);
    double bT = 2.0 * kap1 * kap2 / (dz2 * kap1 + dz1 * kap2);
    r.sigma_xz = bu * (u2 - u1);
    r.pi_z = -bT * (T2 - T1);
    r.uw1 = u1 + r.sigma_xz * dz1 / (2.0 * mu1);
    r.uw2 = u2 - r.sigma_xz * dz2 / (2.0 * mu2);
    r.tw1 = T1 - r.pi_z * dz1 / (2.0 * kap1);
    r.tw2 = T2 + r.pi_z * dz2 / (2.0 * kap2);
    return r;
}

static double kappa_of(double mu, double gamma, double prandtl)
{
    /* kappa = mu c_p / Pr with nondimensional c_p = 1/(gamma-1) (App. A). */
    return mu / ((gamma - 1.0) * prandtl);
}

/* ------------------------------------------------------------------------ */
/* One domain's semi-discrete RHS (eq. cns-fv in the Cartesian form of      */
/* Appendix B, eq. ns-fv-cartesian-3d, restricted to x-z) on rows           */
/* [k_lo, k_hi).  Boundaries: 'bot_gamma' / 'top_gamma' select the rigid    */
/* lid below / above; otherwise a slip adiabatic wall.  fvg is the per-     */
/* column interface viscous flux (4 components, +z direction).              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nx, nz;
    double dx, dz, mu, kappa, gamma, gravity;
    int bot_gamma, top_gamma;
} dom_t;

static void domain_rhs(const dom_t* D, const double* q, const double* fvg,
                       double* r, int k_lo, int k_hi)
{
    const int nx = D->nx, nz = D->nz;
    const int ne = nz + 2; /* extended rows: -1 .. nz */
    const double gm = D->gamma;
    if (k_lo < 0) k_lo = 0;
    if (k_hi > nz) k_hi = nz;
    if (k_lo >= k_hi) return;

    /* Extended conserved state with mirror ghost rows (row e = k + 1). */
    double* qe = (double*)malloc(sizeof(double) * NV * (size_t)ne * nx);
    double* ue = (double*)malloc(sizeof(double) * (size_t)ne * nx);
    double* we = (double*)malloc(sizeof(double) * (size_t)ne * nx);
    double* Te = (double*)malloc(sizeof(double) * (size_t)ne * nx);
    /* Cell gradients (central differences; the least-squares gradient on a
     * uniform grid, Appendix B footnote), on interior rows only. */
    double* dqx = (double*)malloc(sizeof(double) * NV * (size_t)nz * nx);
    double* dqz = (double*)malloc(sizeof(double) * NV * (size_t)nz * nx);
    double* dux = (double*)malloc(sizeof(double) * (size_t)nz * nx);
    double* duz = (double*)malloc(sizeof(double) * (size_t)nz * nx);
    double* dwx = (double*)malloc(sizeof(double) * (size_t)nz * nx);
    double* dwz = (double*)malloc(sizeof(double) * (size_t)nz * nx);
    /* Face fluxes: x-faces i+1/2 for each row, z-faces below row f (f = 0
     * is the bottom boundary, f = nz the top boundary). */
    double* Fx = (double*)malloc(sizeof(double) * NV * (size_t)nz * nx);
    double* Fz = (double*)malloc(sizeof(double) * NV * (size_t)(nz + 1) * nx);

#pragma omp parallel for schedule(static) if (par_ok((size_t)nx * nz))
    for (int e = 0; e < ne; ++e) {
        int k = e - 1;
        int src = k < 0 ? 0 : (k >= nz ? nz - 1 : k);
        int ghost = (k < 0 || k >= nz);
        for (int i = 0; i < nx; ++i) {
            double c[NV], g[NV];
            for (int v = 0; v < NV; ++v) c[v] = q[at(nx, nz, v, src, i)];
            if (ghost) mirror(c, g); else memcpy(g, c, sizeof g);
            for (int v = 0; v < NV; ++v) qe[at(nx, ne, v, e, i)] = g[v];
            double p = pressure(g, gm);
            ue[(size_t)e * nx + i] = g[I_MX] / g[I_RHO];
            we[(size_t)e * nx + i] = g[I_MZ] / g[I_RHO];
            Te[(size_t)e * nx + i] = gm * p / g[I_RHO];
        }
    }

#pragma omp parallel for schedule(static) if (par_ok((size_t)nx * nz))
    for (int k = 0; k < nz; ++k) {
        int e = k + 1;
        for (int i = 0; i < nx; ++i) {
            int im = wrap(i - 1, nx), ip = wrap(i + 1, nx);
            for (int v = 0; v < NV; ++v) {
                dqx[at(nx, nz, v, k, i)] =
                    (qe[at(nx, ne, v, e, ip)] - qe[at(nx, ne, v, e, im)]) / (2.0 * D->dx);
                dqz[at(nx, nz, v, k, i)] =
                    (qe[at(nx, ne, v, e + 1, i)] - qe[at(nx, ne, v, e - 1, i)]) / (2.0 * D->dz);
            }
            size_t c = (size_t)k * nx + i;
            dux[c] = (ue[(size_t)e * nx + ip] - ue[(size_t)e * nx + im]) / (2.0 * D->dx);
            dwx[c] = (we[(size_t)e * nx + ip] - we[(size_t)e * nx + im]) / (2.0 * D->dx);
            duz[c] = (ue[(size_t)(e + 1) * nx + i] - ue[(size_t)(e - 1) * nx + i]) / (2.0 * D->dz);
            dwz[c] = (we[(size_t)(e + 1) * nx + i] - we[(size_t)(e - 1) * nx + i]) / (2.0 * D->dz);
        }
    }

    /* x-faces on the requested rows. */
#pragma omp parallel for schedule(static) if (par_ok((size_t)nx * nz))
    for (int k = k_lo; k < k_hi; ++k) {
        int e = k + 1;
        for (int i = 0; i < nx; ++i) {
            int ip = wrap(i + 1, nx);
            double qL[NV], qR[NV], F[NV];
            for (int v = 0; v < NV; ++v) {
                qL[v] = qe[at(nx, ne, v, e, i)] + dqx[at(nx, nz, v, k, i)] * (D->dx / 2.0);
                qR[v] = qe[at(nx, ne, v, e, ip)] - dqx[at(nx, nz, v, k, ip)] * (D->dx / 2.0);
            }
            llf_flux(qL, qR, 0, gm, F);
            /* Common values (Appendix B): average velocity, normal gradient
             * by finite difference, tangential gradient by averaging. */
            size_t cL = (size_t)e * nx + i, cR = (size_t)e * nx + ip;
            double uh = 0.5 * (ue[cL] + ue[cR]);
            double wh = 0.5 * (we[cL] + we[cR]);
            double ux = (ue[cR] - ue[cL]) / D->dx;
            double wx = (we[cR] - we[cL]) / D->dx;
            double Tx = (Te[cR] - Te[cL]) / D->dx;
            double uz = 0.5 * (duz[(size_t)k * nx + i] + duz[(size_t)k * nx + ip]);
            double wz = 0.5 * (dwz[(size_t)k * nx + i] + dwz[(size_t)k * nx + ip]);
            double sxx = D->mu * (4.0 / 3.0 * ux - 2.0 / 3.0 * wz);
            double sxz = D->mu * (uz + wx);
            double fv[NV] = {0.0, sxx, sxz, uh * sxx + wh * sxz + D->kappa * Tx};
            for (int v = 0; v < NV; ++v) Fx[at(nx, nz, v, k, i)] = F[v] - fv[v];
        }
    }

    /* z-faces f = k_lo .. k_hi (below row f). */
#pragma omp parallel for schedule(static) if (par_ok((size_t)nx * nz))
    for (int f = k_lo; f <= k_hi; ++f) {
        for (int i = 0; i < nx; ++i) {
            double qL[NV], qR[NV], F[NV], fv[NV] = {0.0, 0.0, 0.0, 0.0};
            if (f == 0 || f == nz) {
                /* Boundary face: reconstructed interior state and its mirror. */
                int k = (f == 0) ? 0 : nz - 1;
                double qh[NV];
                double sgn = (f == 0) ? -1.0 : 1.0;
                for (int v = 0; v < NV; ++v)
                    qh[v] = q[at(nx, nz, v, k, i)] + sgn * dqz[at(nx, nz, v, k, i)] * (D->dz / 2.0);
                if (f == 0) { mirror(qh, qL); memcpy(qR, qh, sizeof qR); }
                else        { memcpy(qL, qh, sizeof qL); mirror(qh, qR); }
                llf_flux(qL, qR, 1, gm, F);
                int is_gamma = (f == 0) ? D->bot_gamma : D->top_gamma;
                if (is_gamma)
                    for (int v = 0; v < NV; ++v) fv[v] = fvg[(size_t)i * NV + v];
            } else {
                int kl = f - 1, kr = f;
                for (int v = 0; v < NV; ++v) {
                    qL[v] = q[at(nx, nz, v, kl, i)] + dqz[at(nx, nz, v, kl, i)] * (D->dz / 2.0);
                    qR[v] = q[at(nx, nz, v, kr, i)] - dqz[at(nx, nz, v, kr, i)] * (D->dz / 2.0);
                }
                llf_flux(qL, qR, 1, gm, F);
                size_t cL = (size_t)(kl + 1) * nx + i, cR = (size_t)(kr + 1) * nx + i;
                double uh = 0.5 * (ue[cL] + ue[cR]);
                double wh = 0.5 * (we[cL] + we[cR]);
                double uz = (ue[cR] - ue[cL]) / D->dz;
                double wz = (we[cR] - we[cL]) / D->dz;
                double Tz = (Te[cR] - Te[cL]) / D->dz;
                double ux = 0.5 * (dux[(size_t)kl * nx + i] + dux[(size_t)kr * nx + i]);
                double wx = 0.5 * (dwx[(size_t)kl * nx + i] + dwx[(size_t)kr * nx + i]);
                double szx = D->mu * (uz + wx);
                double szz = D->mu * (4.0 / 3.0 * wz - 2.0 / 3.0 * ux);
                fv[1] = szx;
                fv[2] = szz;
                fv[3] = uh * szx + wh * szz + D->kappa * Tz;
            }
            for (int v = 0; v < NV; ++v) Fz[at(nx, nz + 1, v, f, i)] = F[v] - fv[v];
        }
    }

    /* Divergence plus source. */
#pragma omp parallel for schedule(static) if (par_ok((size_t)nx * nz))
    for (int k = k_lo; k < k_hi; ++k) {
        for (int i = 0; i < nx; ++i) {
            int im = wrap(i - 1, nx);
            double rho = q[at(nx, nz, I_RHO, k, i)];
            double mz = q[at(nx, nz, I_MZ, k, i)];
            double src[NV] = {0.0, 0.0, rho * D->gravity, mz * D->gravity};
            for (int v = 0; v < NV; ++v) {
                double dfx = (Fx[at(nx, nz, v, k, i)] - Fx[at(nx, nz, v, k, im)]) / D->dx;
                double dfz = (Fz[at(nx, nz + 1, v, k + 1, i)] - Fz[at(nx, nz + 1, v, k, i)]) / D->dz;
                r[at(nx, nz, v, k, i)] = -dfx - dfz + src[v];
            }
        }
    }

    free(qe); free(ue); free(we); free(Te);
    free(dqx); free(dqz); free(dux); free(duz); free(dwx); free(dwz);
    free(Fx); free(Fz);
}

static void make_domains(const orc_cfg* c, dom_t* lo, dom_t* up)
{
    lo->nx = c->nx; lo->nz = c->nz_lower; lo->dx = c->dx; lo->dz = c->dz_lower;
    lo->mu = c->mu_lower; lo->kappa = kappa_of(c->mu_lower, c->gamma, c->prandtl);
    lo->gamma = c->gamma; lo->gravity = c->gravity; lo->bot_gamma = 0; lo->top_gamma = 1;
    up->nx = c->nx; up->nz = c->nz_upper; up->dx = c->dx; up->dz = c->dz_upper;
    up->mu = c->mu_upper; up->kappa = kappa_of(c->mu_upper, c->gamma, c->prandtl);
    up->gamma = c->gamma; up->gravity = c->gravity; up->bot_gamma = 1; up->top_gamma = 0;
}

/* Cell-average primitive u and T of one cell. */
static void cell_uT(const double* q, int nx, int nz, int k, int i, double gamma,
                    double* u, double* T)
{
    double c[NV];
    for (int v = 0; v < NV; ++v) c[v] = q[at(nx, nz, v, k, i)];
    *u = c[I_MX] / c[I_RHO];
    *T = gamma * pressure(c, gamma) / c[I_RHO];
}

/* Per-column interface quantities from the two cells next to Gamma. */
static void interface_all(const orc_cfg* c, const double* qlo, const double* qup,
                          iface_t* out)
{
    double kl = kappa_of(c->mu_lower, c->gamma, c->prandtl);
    double ku = kappa_of(c->mu_upper, c->gamma, c->prandtl);
    for (int i = 0; i < c->nx; ++i) {
        double u1, T1, u2, T2;
        cell_uT(qlo, c->nx, c->nz_lower, c->nz_lower - 1, i, c->gamma, &u1, &T1);
        cell_uT(qup, c->nx, c->nz_upper, 0, i, c->gamma, &u2, &T2);
        out[i] = interface_column(u1, T1, u2, T2, c->mu_lower, c->mu_upper, kl, ku,
                                  c->dz_lower, c->dz_upper);
    }
}

/* Coupled RHS on the requested rows of each domain (rows outside the ranges
 * are left untouched in r_lo / r_up). */
static void coupled_rhs(const orc_cfg* c, const double* qlo, const double* qup,
                        double* rlo, double* rup, int lo0, int hi0, int lo1, int hi1)
{
    dom_t L, U;
    make_domains(c, &L, &U);
    iface_t* ifc = (iface_t*)malloc(sizeof(iface_t) * (size_t)c->nx);
    double* fvg = (double*)malloc(sizeof(double) * NV * (size_t)c->nx);
    interface_all(c, qlo, qup, ifc);
    for (int i = 0; i < c->nx; ++i) {
        /* hat w = 0 and hat sigma_zz = 0 on the lid, so the +z viscous flux
         * is (0, sigma_xz, 0, u_w sigma_xz - Pi_z). */
        fvg[(size_t)i * NV + 0] = 0.0;
        fvg[(size_t)i * NV + 1] = ifc[i].sigma_xz;
        fvg[(size_t)i * NV + 2] = 0.0;
        fvg[(size_t)i * NV + 3] = ifc[i].uw1 * ifc[i].sigma_xz - ifc[i].pi_z;
    }
    domain_rhs(&L, qlo, fvg, rlo, lo0, hi0);
    domain_rhs(&U, qup, fvg, rup, lo1, hi1);
    free(ifc);
    free(fvg);
}

/* ======================================================================== */
/* Exported API                                                              */
/* ======================================================================== */

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Full coupled RHS of both domains (all rows). */
int orc_rhs(const orc_cfg* c, const double* qlo, const double* qup, double* rlo, double* rup)
{
    coupled_rhs(c, qlo, qup, rlo, rup, 0, c->nz_lower, 0, c->nz_upper);
    return 0;
}

/* Coupled RHS restricted to row ranges. */
int orc_rhs_rows(const orc_cfg* c, const double* qlo, const double* qup, double* rlo,
                 double* rup, int lo0, int hi0, int lo1, int hi1)
{
    coupled_rhs(c, qlo, qup, rlo, rup, lo0, hi0, lo1, hi1);
    return 0;
}

/* Per-column interface quantities: out[i*6 + {0..5}] = sigma_xz, Pi_z, u_w1,
 * u_w2, T_w1, T_w2. */
int orc_interface(const orc_cfg* c, const double* qlo, const double* qup, double* out)
{
    iface_t* ifc = (iface_t*)malloc(sizeof(iface_t) * (size_t)c->nx);
    interface_all(c, qlo, qup, ifc);
    for (int i = 0; i < c->nx; ++i) {
        out[i * 6 + 0] = ifc[i].sigma_xz;
        out[i * 6 + 1] = ifc[i].pi_z;
        out[i * 6 + 2] = ifc[i].uw1;
        out[i * 6 + 3] = ifc[i].uw2;
        out[i * 6 + 4] = ifc[i].tw1;
        out[i * 6 + 5] = ifc[i].tw2;
    }
    free(ifc);
    return 0;
}

/* LLF flux of two states (exposed for the consistency pins). */
int orc_llf(const double* qL, const double* qR, int dir, double gamma, double* F)
{
    llf_flux(qL, qR, dir, gamma, F);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Base methods and the MPRK tableaux.                                       */
/* base 2: the RK2 base of Table 1 (A21 = 1, b = (1/2, 1/2), c = (0, 1)).   */
/* base 3: three-stage strong-stability-preserving RK3 (A21 = 1, A31 = A32  */
/*         = 1/4, b = (1/6, 1/6, 2/3), c = (0, 1, 1/2)).                    */
/* ------------------------------------------------------------------------ */
static int base_tableau(int base, double* A, double* b, double* cc)
{
    if (base == 2) {
        double a2[4] = {0, 0, 1, 0};
        double b2[2] = {0.5, 0.5}, c2[2] = {0.0, 1.0};
        memcpy(A, a2, sizeof a2); memcpy(b, b2, sizeof b2); memcpy(cc, c2, sizeof c2);
        return 2;
    }
    if (base == 3) {
        double a3[9] = {0, 0, 0, 1, 0, 0, 0.25, 0.25, 0};
        double b3[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0}, c3[3] = {0.0, 1.0, 0.5};
        memcpy(A, a3, sizeof a3); memcpy(b, b3, sizeof b3); memcpy(cc, c3, sizeof c3);
        return 3;
    }
    return -1;
}

/*
 * Expanded ms-stage tableaux of the three partitions (Section 3, eq. MRK2 and
 * Table 1), global stage i = (k-1)s + j for substep k = 1..m and base stage
 * j = 1..s:
 *  F: m substeps of size dt/m.  a_F[(k-1)s+j][(l-1)s+p] = b_p/m for l < k,
 *     A_jp/m for l = k; b_F = b_j/m; c_F = (k-1+c_j)/m.
 *  B: each substep restarts from q_n with the full step:
 *     a_B[(k-1)s+j][(k-1)s+p] = A_jp; b_B = b_j/m; c_B = c_j.
 *  S: one base step; its stage j is reused at every substep:
 *     a_S[(k-1)s+j][p] = A_jp (p <= s); b_S = (b, 0, ..., 0); c_S = c_j.
 * Arrays are row-major ms x ms (a) and ms (b, c).  Returns s, or -1.
 */
int orc_tableau(int base, int m, double* aF, double* bF, double* cF, double* aB,
                double* bB, double* cB, double* aS, double* bS, double* cS)
{
    double A[9], b[3], cc[3];
    int s = base_tableau(base, A, b, cc);
    if (s < 0 || m < 1) return -1;
    int ms = m * s;
    memset(aF, 0, sizeof(double) * ms * ms);
    memset(aB, 0, sizeof(double) * ms * ms);
    memset(aS, 0, sizeof(double) * ms * ms);
    for (int k = 0; k < m; ++k) {
        for (int j = 0; j < s; ++j) {
            int i = k * s + j;
            for (int l = 0; l <= k; ++l)
                for (int p = 0; p < s; ++p)
                    aF[i * ms + l * s + p] = (l < k) ? b[p] / m : A[j * s + p] / m;
            for (int p = 0; p < s; ++p) aB[i * ms + k * s + p] = A[j * s + p];
            for (int p = 0; p < s; ++p) aS[i * ms + p] = A[j * s + p];
            bF[i] = b[j] / m;
            bB[i] = b[j] / m;
            bS[i] = (k == 0) ? b[j] : 0.0;
            cF[i] = (k + cc[j]) / m;
            cB[i] = cc[j];
            cS[i] = cc[j];
        }
    }
    return s;
}

/* Rows of the slow domain that form the buffer B (next to Gamma). */
static void slow_partition(const orc_cfg* c, int* b_lo, int* b_hi)
{
    if (c->fast_is_lower) { *b_lo = 0; *b_hi = c->n_buffer; }
    else { *b_lo = c->nz_lower - c->n_buffer; *b_hi = c->nz_lower; }
}

/*
 * One MPRK step in Butcher form, following Algorithm 1: for each global stage
 * i = 1..ms, form the buffer stage value, the slow stage value (i <= s) or a
 * copy of slow stage mod(i-1,s)+1, and the fast stage value (eq. MRK2-qi);
 * then the RHS of B, of S (i <= s) and of F on the assembled coupled state.
 * Completion by eq. MRK2-qn.  q_lo and q_up are updated in place.
 */
int orc_mprk_step(const orc_cfg* c, int base, int m, double dt, double* qlo, double* qup)
{
    double A[9], bb[3], cc[3];
    int s = base_tableau(base, A, bb, cc);
    if (s < 0 || m < 1) return -1;
    const int ms = m * s, nx = c->nx;
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

    double* qF = c->fast_is_lower ? qlo : qup;
    double* qSl = c->fast_is_lower ? qup : qlo;
    const int nzF = c->fast_is_lower ? c->nz_lower : c->nz_upper;
    const int nzS = c->fast_is_lower ? c->nz_upper : c->nz_lower;
    int b_lo, b_hi;
    slow_partition(c, &b_lo, &b_hi);
    const size_t nF = (size_t)NV * nzF * nx, nS = (size_t)NV * nzS * nx;

    double* RF = (double*)calloc((size_t)ms * nF, sizeof(double));
    double* RS = (double*)calloc((size_t)ms * nS, sizeof(double)); /* slow-domain RHS */
    double* QF = (double*)malloc(sizeof(double) * nF);
    double* QS = (double*)malloc(sizeof(double) * nS);
    double* Ssave = (double*)malloc(sizeof(double) * (size_t)s * nS); /* Q^S_j, j <= s */

    for (int i = 0; i < ms; ++i) {
        /* Buffer rows and slow rows of the slow domain. */
#pragma omp parallel for schedule(static) if (par_ok((size_t)nx * (nzF + nzS)))
        for (int k = 0; k < nzS; ++k) {
            int in_b = (k >= b_lo && k < b_hi);
            for (int v = 0; v < NV; ++v)
                for (int x = 0; x < nx; ++x) {
                    size_t id = at(nx, nzS, v, k, x);
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
                        QS[id] = Ssave[(size_t)(i % s) * nS + id]; /* copy line */
                    }
                }
        }
        /* Fast partition. */
#pragma omp parallel for schedule(static) if (par_ok((size_t)nx * (nzF + nzS)))
        for (int k = 0; k < nzF; ++k)
            for (int v = 0; v < NV; ++v)
                for (int x = 0; x < nx; ++x) {
                    size_t id = at(nx, nzF, v, k, x);
                    double acc = 0.0;
                    for (int j = 0; j < i; ++j) acc += aF[i * ms + j] * RF[(size_t)j * nF + id];
                    QF[id] = qF[id] + dt * acc;
                }

        /* RHS: F everywhere, B always, S only at the first s stages. */
        int s_lo = (i < s) ? 0 : b_lo, s_hi = (i < s) ? nzS : b_hi;
        double* rF = RF + (size_t)i * nF;
        double* rS = RS + (size_t)i * nS;
        if (c->fast_is_lower)
            coupled_rhs(c, QF, QS, rF, rS, 0, nzF, s_lo, s_hi);
        else
            coupled_rhs(c, QS, QF, rS, rF, s_lo, s_hi, 0, nzF);
    }

    /* Completion, eq. MRK2-qn. */
#pragma omp parallel for schedule(static) if (par_ok((size_t)nx * (nzF + nzS)))
    for (int k = 0; k < nzF; ++k)
        for (int v = 0; v < NV; ++v)
            for (int x = 0; x < nx; ++x) {
                size_t id = at(nx, nzF, v, k, x);
                double acc = 0.0;
                for (int i = 0; i < ms; ++i) acc += bF[i] * RF[(size_t)i * nF + id];
                qF[id] = qF[id] + dt * acc;
            }
#pragma omp parallel for schedule(static) if (par_ok((size_t)nx * (nzF + nzS)))
    for (int k = 0; k < nzS; ++k) {
        int in_b = (k >= b_lo && k < b_hi);
        for (int v = 0; v < NV; ++v)
            for (int x = 0; x < nx; ++x) {
                size_t id = at(nx, nzS, v, k, x);
                double acc = 0.0;
                if (in_b) {
                    for (int i = 0; i < ms; ++i) acc += bB[i] * RS[(size_t)i * nS + id];
                } else {
                    for (int i = 0; i < s; ++i) acc += bS[i] * RS[(size_t)i * nS + id];
                }
                qSl[id] = qSl[id] + dt * acc;
            }
    }

    free(aF); free(aB); free(aS); free(bF); free(bB); free(bS);
    free(cF); free(cB); free(cS);
    free(RF); free(RS); free(QF); free(QS); free(Ssave);
    return 0;
}

/*
 * One single-rate step of the base method on the whole coupled state,
 * coded independently of orc_mprk_step (used to check that MPRK with m = 1
 * is the base method).
 */
int orc_sr_step(const orc_cfg* c, int base, double dt, double* qlo, double* qup)
{
    double A[9], b[3], cc[3];
    int s = base_tableau(base, A, b, cc);
    if (s < 0) return -1;
    const size_t nL = (size_t)NV * c->nz_lower * c->nx, nU = (size_t)NV * c->nz_upper * c->nx;
    double* RL = (double*)calloc((size_t)s * nL, sizeof(double));
    double* RU = (double*)calloc((size_t)s * nU, sizeof(double));
    double* QL = (double*)malloc(sizeof(double) * nL);
    double* QU = (double*)malloc(sizeof(double) * nU);
    for (int i = 0; i < s; ++i) {
        for (size_t id = 0; id < nL; ++id) {
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc += A[i * s + j] * RL[(size_t)j * nL + id];
            QL[id] = qlo[id] + dt * acc;
        }
        for (size_t id = 0; id < nU; ++id) {
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc += A[i * s + j] * RU[(size_t)j * nU + id];
            QU[id] = qup[id] + dt * acc;
        }
        orc_rhs(c, QL, QU, RL + (size_t)i * nL, RU + (size_t)i * nU);
    }
    for (size_t id = 0; id < nL; ++id) {
        double acc = 0.0;
        for (int i = 0; i < s; ++i) acc += b[i] * RL[(size_t)i * nL + id];
        qlo[id] = qlo[id] + dt * acc;
    }
    for (size_t id = 0; id < nU; ++id) {
        double acc = 0.0;
        for (int i = 0; i < s; ++i) acc += b[i] * RU[(size_t)i * nU + id];
        qup[id] = qup[id] + dt * acc;
    }
    free(RL); free(RU); free(QL); free(QU);
    return 0;
}

/* n MPRK steps (m = 1 is the base method through the MPRK code path). */
int orc_mprk_run(const orc_cfg* c, int base, int m, double dt, int64_t n, double* qlo, double* qup)
{
    for (int64_t t = 0; t < n; ++t) {
        int rc = orc_mprk_step(c, base, m, dt, qlo, qup);
        if (rc) return rc;
    }
    return 0;
}

int orc_sr_run(const orc_cfg* c, int base, double dt, int64_t n, double* qlo, double* qup)
{
    for (int64_t t = 0; t < n; ++t) {
        int rc = orc_sr_step(c, base, dt, qlo, qup);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                              */
/* ------------------------------------------------------------------------ */

/* Neumaier-compensated sum of q over one domain, times the cell measure
 * (total mass / momentum / energy as in Section 5.1). */
static double total_of(const double* q, int nx, int nz, int v, double area)
{
    double s = 0.0, comp = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
            double x = q[at(nx, nz, v, k, i)];
            double t = s + x;
            if (fabs(s) >= fabs(x)) comp += (s - t) + x;
            else comp += (x - t) + s;
            s = t;
        }
    return (s + comp) * area;
}

/* totals[0..3] lower domain, totals[4..7] upper domain. */
int orc_totals(const orc_cfg* c, const double* qlo, const double* qup, double* totals)
{
    for (int v = 0; v < NV; ++v) {
        totals[v] = total_of(qlo, c->nx, c->nz_lower, v, c->dx * c->dz_lower);
        totals[NV + v] = total_of(qup, c->nx, c->nz_upper, v, c->dx * c->dz_upper);
    }
    return 0;
}

/*
 * Per-domain stability measures.  lam[d] = max over cells of the directional
 * sum (|u|+a)/dx + (|w|+a)/dz (the multi-dimensional Courant measure used by
 * the step-size rule); cour[d] = max over cells and directions of
 * (|u_dir|+a)/d_dir (the Courant number printed in the paper's tables is
 * dt * cour); vis[d] = max over cells of max(4/3, gamma/Pr) mu_d / rho *
 * (1/dx^2 + 1/dz^2).  Returns 1 if any value is non-finite, rho <= 0 or
 * p <= 0.
 */
int orc_wave_measures(const orc_cfg* c, const double* qlo, const double* qup, double* lam,
                      double* cour, double* vis)
{
    int bad = 0;
    for (int d = 0; d < 2; ++d) {
        const double* q = d == 0 ? qlo : qup;
        int nz = d == 0 ? c->nz_lower : c->nz_upper;
        double dz = d == 0 ? c->dz_lower : c->dz_upper;
        double mu = d == 0 ? c->mu_lower : c->mu_upper;
        double coef = 4.0 / 3.0;
        if (c->gamma / c->prandtl > coef) coef = c->gamma / c->prandtl;
        double L = 0.0, C = 0.0, V = 0.0;
        for (int k = 0; k < nz; ++k)
            for (int i = 0; i < c->nx; ++i) {
                double cc[NV];
                for (int v = 0; v < NV; ++v) cc[v] = q[at(c->nx, nz, v, k, i)];
                double p = pressure(cc, c->gamma);
                if (!(cc[I_RHO] > 0.0) || !(p > 0.0) || !isfinite(cc[I_MX]) ||
                    !isfinite(cc[I_MZ]) || !isfinite(cc[I_EN])) {
                    bad = 1;
                    continue;
                }
                double a = sqrt(c->gamma * p / cc[I_RHO]);
                double sx = (fabs(cc[I_MX] / cc[I_RHO]) + a) / c->dx;
                double sz = (fabs(cc[I_MZ] / cc[I_RHO]) + a) / dz;
                if (sx + sz > L) L = sx + sz;
                if (sx > C) C = sx;
                if (sz > C) C = sz;
                double vv = coef * mu / cc[I_RHO] * (1.0 / (c->dx * c->dx) + 1.0 / (dz * dz));
                if (vv > V) V = vv;
            }
        lam[d] = L;
        cour[d] = C;
        vis[d] = V;
    }
    return bad;
}

/*
 * Step-size rule.  Per domain the stable step is 1 / (lam/cr + vis/dn): the
 * advective (Courant) and diffusive (viscous and heat-conduction) limits are
 * combined, because the odd-even mode receives both as negative real
 * eigenvalue contributions (upwind-type dissipation 2 lam, diffusion 4 vis),
 * so their sum must stay inside the real-axis stability interval.  Fast
 * step dt_f from the fast domain; slow step dt = min(m dt_f, slow-domain
 * step).  Returns dt (0 on a bad state).
 */
static double domain_step(double lam, double vis, double cr, double dn)
{
    return 1.0 / (lam / cr + vis / dn);
}

double orc_dt_rule(const orc_cfg* c, const double* qlo, const double* qup, int m, double cr,
                   double dn)
{
    double lam[2], cour[2], vis[2];
    if (orc_wave_measures(c, qlo, qup, lam, cour, vis)) return 0.0;
    int f = c->fast_is_lower ? 0 : 1, sl = 1 - f;
    double dtf = domain_step(lam[f], vis[f], cr, dn);
    double dts = domain_step(lam[sl], vis[sl], cr, dn);
    double dt = m * dtf;
    if (dts < dt) dt = dts;
    return dt;
}
