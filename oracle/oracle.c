/*
 * oracle.c -- plain, slow, FP64 CPU reference of the adaptive finite-volume
 * method for the compressible Euler equations (ideal gas, Cartesian 2D/3D)
 * of Deiterding, Domingues, Gomes and Schneider, "Comparison of adaptive
 * multiresolution and adaptive mesh refinement applied to simulations of the
 * compressible Euler equations" (arXiv:1603.05211).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library and includes nothing of it.
 *
 * Every routine is written for a reader to check against the paper by eye:
 * one cell at a time, FP64 throughout, no blocking, no fusion.  Loops over
 * independent cells carry an OpenMP pragma; every output cell is computed by
 * the same expression whatever the thread count, so results do not depend
 * on it.  Build with -O2 -ffp-contract=off (no FMA contraction).
 *
 * Layout: level l holds a dense grid of n_l^d cells, n_l = n0 * 2^l.  The
 * conserved fields (rho, m_1..m_d, E) are stored one after another, x fastest:
 *     Q[f * n^d + x + n * (y + n * z)]          (z = 0 in 2D).
 * Cells of a level that belong to no refinement patch still have storage;
 * they are read only where they are ghost cells (filled by prediction).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXL 10
#define NVMAX 5

enum { BC_TRANSMISSIVE = 0, BC_PERIODIC = 1 };

/* Test-only planted mistakes (controls that show a pin can fail): 0 = none;
 * 1 = AUSM+ without its alpha / beta terms (plain AUSM splitting);
 * 2 = the z pass of the 3D prediction with the upper / lower child swapped;
 * 3 = ghost cells of local time stepping taken from the coarse state at the
 *     start of its step at every stage (constant theta = 0);
 * 4 = AUSMDV with its pressure-ratio weights alpha_L = alpha_R = 1;
 * 5 = MUSCL-Hancock without the half-step evolution of the face states;
 * 6 = a leaf next to a covered cell takes its own level's flux at that face
 *     instead of the mean of the finer level's fluxes (global time step).
 * With 0 every result is the method's, bit for bit. */
enum { PLANT_NONE = 0, PLANT_AUSM_AB = 1, PLANT_PRED_ZSWAP = 2, PLANT_LTS_THETA = 3,
       PLANT_AUSMDV_ALPHA = 4, PLANT_HANCOCK_NOPRED = 5, PLANT_NO_FINE_MEAN = 6 };
static int plant = PLANT_NONE;
void orc_set_plant(int which) { plant = which; }

/* ------------------------------------------------------------------------ */
/* grid helpers                                                             */
/* ------------------------------------------------------------------------ */

/* Ghost index map for the physical boundary.  Outflow (transmissive) takes
 * the nearest interior cell (zero-order extrapolation); periodic wraps.
 * Sec. 4.1 / 4.2: outflow conditions at all sides of the domain. */
static int bcmap(int i, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        i %= n;
        if (i < 0) i += n;
        return i;
    }
    if (i < 0) return 0;
    if (i >= n) return n - 1;
    return i;
}

static int64_t ncells(int dim, int n)
{
    return dim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
}

static int64_t cidx(int n, const int *c)
{
    return c[0] + (int64_t)n * (c[1] + (int64_t)n * c[2]);
}

static void cdecode(int dim, int n, int64_t i, int *c)
{
    c[0] = (int)(i % n);
    c[1] = (int)((i / n) % n);
    c[2] = dim == 3 ? (int)(i / ((int64_t)n * n)) : 0;
}

/* ------------------------------------------------------------------------ */
/* physics: Sec. 2, conservation law, fluxes f_1..f_3 and ideal-gas relation */
/* ------------------------------------------------------------------------ */

/* conserved (rho, rho v, rho e) -> primitive (rho, v, p);
 * p = (gamma - 1) (rho e - rho |v|^2 / 2). */
static void cons2prim(int dim, double g, const double *q, double *w)
{
    double rho = q[0], K = 0.0;
    w[0] = rho;
    for (int d = 0; d < dim; ++d) {
        double v = q[1 + d] / rho;
        w[1 + d] = v;
        K = K + v * v;
    }
    w[dim + 1] = (g - 1.0) * (q[dim + 1] - (0.5 * rho) * K);
}

/* primitive -> conserved; rho e = p / (gamma - 1) + rho |v|^2 / 2. */
static void prim2cons(int dim, double g, const double *w, double *q)
{
    double rho = w[0], K = 0.0, gi = 1.0 / (g - 1.0);
    q[0] = rho;
    for (int d = 0; d < dim; ++d) {
        q[1 + d] = rho * w[1 + d];
        K = K + w[1 + d] * w[1 + d];
    }
    q[dim + 1] = w[dim + 1] * gi + (0.5 * rho) * K;
}

/* van Albada limited slope of the MUSCL reconstruction (Sec. 2, MR scheme),
 * in slope form: sigma = a b (a + b) / (a^2 + b^2) for a b > 0, else 0,
 * with a, b the backward and forward differences. */
static double slope_va(double wm, double w0, double wp)
{
    double a = w0 - wm, b = wp - w0, ab = a * b;
    if (ab > 0.0) return (ab * (a + b)) / (a * a + b * b);
    return 0.0;
}

/* AUSM+ flux-vector splitting (Liou 1996; Sec. 2, MR scheme) across a face
 * with normal along axis dn.  wL / wR are the primitive face states.
 * Interface sound speed (speed): 0 the arithmetic mean of the two sound
 * speeds (the default); 1 Liou's critical speed, c_1/2 =
 * min(c*_L^2 / max(c*_L, u_L), c*_R^2 / max(c*_R, -u_R)) with c*^2 =
 * 2 (gamma - 1) / (gamma + 1) H, H the total enthalpy (a variant).
 * alpha = 3/16, beta = 1/8. */
static void ausm_plus(int dim, double g, int dn, const double *wL,
                      const double *wR, double *F, int speed)
{
    double gi = 1.0 / (g - 1.0);
    double rL = wL[0], pL = wL[dim + 1], uL = wL[1 + dn];
    double rR = wR[0], pR = wR[dim + 1], uR = wR[1 + dn];
    double ch;
    if (speed == 1) {
        double KL = 0.0, KR = 0.0;
        for (int k = 0; k < dim; ++k) {
            KL = KL + wL[1 + k] * wL[1 + k];
            KR = KR + wR[1 + k] * wR[1 + k];
        }
        double HL = ((pL * gi + (0.5 * rL) * KL) + pL) / rL;
        double HR = ((pR * gi + (0.5 * rR) * KR) + pR) / rR;
        double kc = (2.0 * (g - 1.0)) / (g + 1.0);
        double sL = kc * HL, sR = kc * HR;     /* c*^2 */
        double csL = sqrt(sL), csR = sqrt(sR);
        double tL = sL / (csL >= uL ? csL : uL);
        double tR = sR / (csR >= -uR ? csR : -uR);
        ch = tL <= tR ? tL : tR;
    } else {
        double cL = sqrt((g * pL) / rL);
        double cR = sqrt((g * pR) / rR);
        ch = 0.5 * (cL + cR);
    }
    double ML = uL / ch, MR = uR / ch;
    double Mp, Pp, Mm, Pm;
    /* Liou's coefficients alpha = 3/16, beta = 1/8; 16 beta = 2 and
     * 16 alpha = 3 exactly */
    const double alpha = plant == PLANT_AUSM_AB ? 0.0 : 3.0 / 16.0;
    const double beta = plant == PLANT_AUSM_AB ? 0.0 : 1.0 / 8.0;
    const double b16 = 16.0 * beta, a16 = 16.0 * alpha;
    /* split Mach number M4+ and pressure P5+ of the left state */
    if (fabs(ML) >= 1.0) {
        Mp = 0.5 * (ML + fabs(ML));
        Pp = ML > 0.0 ? 1.0 : 0.0;
    } else {
        double a = ML + 1.0, b = ML - 1.0;
        double m2p = 0.25 * (a * a), m2m = -0.25 * (b * b);
        Mp = m2p * (1.0 - b16 * m2m);
        Pp = m2p * ((2.0 - ML) - (a16 * ML) * m2m);
    }
    /* split Mach number M4- and pressure P5- of the right state */
    if (fabs(MR) >= 1.0) {
        Mm = 0.5 * (MR - fabs(MR));
        Pm = MR < 0.0 ? 1.0 : 0.0;
    } else {
        double a = MR + 1.0, b = MR - 1.0;
        double m2p = 0.25 * (a * a), m2m = -0.25 * (b * b);
        Mm = m2m * (1.0 + b16 * m2p);
        Pm = m2m * ((-2.0 - MR) + (a16 * MR) * m2p);
    }
    double mh = Mp + Mm;
    double ph = Pp * pL + Pm * pR;
    double mf = ch * mh;
    const double *wu = mh >= 0.0 ? wL : wR;        /* upwind state */
    double ru = wu[0], pu = wu[dim + 1], K = 0.0;
    for (int k = 0; k < dim; ++k) K = K + wu[1 + k] * wu[1 + k];
    double rH = (pu * gi + (0.5 * ru) * K) + pu;     /* rho e + p */
    F[0] = mf * ru;
    for (int k = 0; k < dim; ++k) {
        F[1 + k] = mf * (ru * wu[1 + k]);
        if (k == dn) F[1 + k] = F[1 + k] + ph;
    }
    F[dim + 1] = mf * rH;
}

/* Numerical flux at the face between cell c (coordinates, axis dn may be
 * outside the domain) and c + e_dn, from the 4-cell stencil c-1 .. c+2 along
 * dn of array A on an n^d grid: primitive MUSCL face states + AUSM+. */
static void face_flux(int dim, int n, int bc, double g, const double *A,
                      int dn, const int *c, double *F, int speed)
{
    int64_t N = ncells(dim, n);
    double w[4][NVMAX], q[NVMAX], wL[NVMAX], wR[NVMAX];
    int nv = dim + 2;
    for (int k = 0; k < 4; ++k) {
        int p[3] = {c[0], c[1], c[2]};
        p[dn] = bcmap(c[dn] + k - 1, n, bc);
        int64_t id = cidx(n, p);
        for (int f = 0; f < nv; ++f) q[f] = A[f * N + id];
        cons2prim(dim, g, q, w[k]);
    }
    for (int f = 0; f < nv; ++f) {
        wL[f] = w[1][f] + 0.5 * slope_va(w[0][f], w[1][f], w[2][f]);
        wR[f] = w[2][f] - 0.5 * slope_va(w[1][f], w[2][f], w[3][f]);
    }
    ausm_plus(dim, g, dn, wL, wR, F, speed);
}

/* ------------------------------------------------------------------------ */
/* the AMR scheme of Sec. 2: unsplit MUSCL-Hancock, Minmod, AUSMDV           */
/* ------------------------------------------------------------------------ */

/* Minmod limited slope: the difference of smaller magnitude when the
 * backward and forward differences have the same sign, else 0. */
static double slope_minmod(double wm, double w0, double wp)
{
    double a = w0 - wm, b = wp - w0;
    if (!(a * b > 0.0)) return 0.0;
    return fabs(a) <= fabs(b) ? a : b;
}

/* Physical flux f_dn of the Euler equations (Sec. 2, the conservation law)
 * at a primitive state w: (rho u, rho u v + p e_dn, u (rho e + p)), u the
 * velocity along dn. */
static void phys_flux(int dim, double g, int dn, const double *w, double *F)
{
    double gi = 1.0 / (g - 1.0);
    double r = w[0], u = w[1 + dn], p = w[dim + 1], K = 0.0;
    for (int k = 0; k < dim; ++k) K = K + w[1 + k] * w[1 + k];
    double E = p * gi + (0.5 * r) * K;
    double m = r * u;
    F[0] = m;
    for (int k = 0; k < dim; ++k) {
        F[1 + k] = m * w[1 + k];
        if (k == dn) F[1 + k] = F[1 + k] + p;
    }
    F[dim + 1] = u * (E + p);
}

/* AUSMDV flux-vector splitting (Wada and Liou 1997, cited in Sec. 2 for the
 * AMR scheme) across a face with normal along axis dn; wL / wR primitive.
 * Common sound speed c_m = max(c_L, c_R); the split velocities blend the
 * AUSM polynomial and the upwind velocity with the pressure-ratio weights
 * alpha = 2 (p/rho) / ((p/rho)_L + (p/rho)_R); third-order pressure
 * polynomials; the normal momentum flux blends the AUSMV form (weight
 * 1/2 + s) and the AUSMD form (1/2 - s), s = min(1, 10 |dp| / min p) / 2;
 * tangential momentum and total enthalpy are upwinded with the mass flux.
 * Plain AUSMDV: neither the entropy fix nor the shock fix. */
static void ausmdv(int dim, double g, int dn, const double *wL,
                   const double *wR, double *F)
{
    double gi = 1.0 / (g - 1.0);
    double rL = wL[0], pL = wL[dim + 1], uL = wL[1 + dn];
    double rR = wR[0], pR = wR[dim + 1], uR = wR[1 + dn];
    double cL = sqrt((g * pL) / rL);
    double cR = sqrt((g * pR) / rR);
    double cm = cL >= cR ? cL : cR;
    double sL = pL / rL, sR = pR / rR;
    double aL = (2.0 * sL) / (sL + sR), aR = (2.0 * sR) / (sL + sR);
    if (plant == PLANT_AUSMDV_ALPHA) aL = aR = 1.0;
    double upL = 0.5 * (uL + fabs(uL)), umR = 0.5 * (uR - fabs(uR));
    double Up, Um, Pp, Pm;
    if (fabs(uL) <= cm) {
        double a = uL + cm, M = uL / cm, b = M + 1.0;
        Up = aL * ((a * a) / (4.0 * cm) - upL) + upL;
        Pp = pL * (((b * b) * (2.0 - M)) * 0.25);
    } else {
        Up = upL;
        Pp = uL > 0.0 ? pL : 0.0;
    }
    if (fabs(uR) <= cm) {
        double a = uR - cm, M = uR / cm, b = M - 1.0;
        Um = aR * (-((a * a) / (4.0 * cm)) - umR) + umR;
        Pm = pR * (((b * b) * (2.0 + M)) * 0.25);
    } else {
        Um = umR;
        Pm = uR < 0.0 ? pR : 0.0;
    }
    double mh = Up * rL + Um * rR;                 /* (rho u)_{1/2} */
    double am = fabs(mh);
    double ph = Pp + Pm;
    double dp = fabs(pR - pL), pmin = pL <= pR ? pL : pR;
    double sw = (10.0 * dp) / pmin;
    double s = 0.5 * (sw < 1.0 ? sw : 1.0);
    double fV = Up * (rL * uL) + Um * (rR * uR);   /* AUSMV normal momentum */
    double fD = 0.5 * (mh * (uL + uR) - am * (uR - uL));   /* AUSMD */
    double KL = 0.0, KR = 0.0;
    for (int k = 0; k < dim; ++k) {
        KL = KL + wL[1 + k] * wL[1 + k];
        KR = KR + wR[1 + k] * wR[1 + k];
    }
    double HL = ((pL * gi + (0.5 * rL) * KL) + pL) / rL;
    double HR = ((pR * gi + (0.5 * rR) * KR) + pR) / rR;
    F[0] = mh;
    for (int k = 0; k < dim; ++k) {
        if (k == dn) F[1 + k] = ((0.5 + s) * fV + (0.5 - s) * fD) + ph;
        else F[1 + k] = 0.5 * (mh * (wL[1 + k] + wR[1 + k]) - am * (wR[1 + k] - wL[1 + k]));
    }
    F[dim + 1] = 0.5 * (mh * (HL + HR) - am * (HR - HL));
}

/* Conserved state at cell position c of array A (positions outside the
 * domain are mapped by the boundary map axis by axis), as primitives. */
static void prim_at(int dim, int n, int bc, double g, const double *A, const int *c, double *w)
{
    int64_t N = ncells(dim, n);
    int p[3] = {bcmap(c[0], n, bc), bcmap(c[1], n, bc), dim == 3 ? bcmap(c[2], n, bc) : 0};
    double q[NVMAX];
    for (int f = 0; f < dim + 2; ++f) q[f] = A[f * N + cidx(n, p)];
    cons2prim(dim, g, q, w);
}

/* MUSCL-Hancock predictor of cell c (Sec. 2, AMR scheme): Minmod slopes of
 * the primitive variables along each axis give the face values
 * W -/+ slope/2; each is advanced half a step in conservative form with the
 * exact flux, dQ = (dt / 2 dx) sum_d [f_d(W^-_d) - f_d(W^+_d)] (summed
 * ((d = 1 + d = 2) + d = 3)), the same increment for every face value of
 * the cell, and returned as primitives Wb[d][0] (lower face of axis d),
 * Wb[d][1] (upper face).  hl = (dt / 2) / dx. */
static void hancock_cell(int dim, int n, int bc, double g, const double *A,
                         const int *c, double hl, double Wb[3][2][NVMAX])
{
    int nv = dim + 2;
    double w0[NVMAX], Wf[3][2][NVMAX], D[3][NVMAX];
    prim_at(dim, n, bc, g, A, c, w0);
    for (int d = 0; d < dim; ++d) {
        double wm[NVMAX], wp[NVMAX];
        int cm[3] = {c[0], c[1], c[2]}, cp[3] = {c[0], c[1], c[2]};
        cm[d] -= 1;
        cp[d] += 1;
        prim_at(dim, n, bc, g, A, cm, wm);
        prim_at(dim, n, bc, g, A, cp, wp);
        for (int f = 0; f < nv; ++f) {
            double sl = slope_minmod(wm[f], w0[f], wp[f]);
            Wf[d][0][f] = w0[f] - 0.5 * sl;
            Wf[d][1][f] = w0[f] + 0.5 * sl;
        }
        double fm[NVMAX], fp[NVMAX];
        phys_flux(dim, g, d, Wf[d][0], fm);
        phys_flux(dim, g, d, Wf[d][1], fp);
        for (int f = 0; f < nv; ++f) D[d][f] = fm[f] - fp[f];
    }
    double dQ[NVMAX];
    for (int f = 0; f < nv; ++f) {
        double S = D[0][f] + D[1][f];
        if (dim == 3) S = S + D[2][f];
        dQ[f] = hl * S;
    }
    for (int d = 0; d < dim; ++d)
        for (int sd = 0; sd < 2; ++sd) {
            double q[NVMAX];
            prim2cons(dim, g, Wf[d][sd], q);
            if (plant != PLANT_HANCOCK_NOPRED)
                for (int f = 0; f < nv; ++f) q[f] = q[f] + dQ[f];
            cons2prim(dim, g, q, Wb[d][sd]);
        }
}

/* AMR-scheme flux at the face between cell c and c + e_dn: AUSMDV of the
 * evolved upper face value of c and lower face value of c + e_dn. */
static void face_flux_hancock(int dim, int n, int bc, double g, const double *A,
                              int dn, const int *c, double hl, double *F)
{
    double Wl[3][2][NVMAX], Wr[3][2][NVMAX];
    int cr[3] = {c[0], c[1], c[2]};
    cr[dn] += 1;
    hancock_cell(dim, n, bc, g, A, c, hl, Wl);
    hancock_cell(dim, n, bc, g, A, cr, hl, Wr);
    ausmdv(dim, g, dn, Wl[dn][1], Wr[dn][0], F);
}

/* ------------------------------------------------------------------------ */
/* multiresolution operators: Sec. 2.1 (projection / prediction, details)    */
/* ------------------------------------------------------------------------ */

/* Projection: a parent's cell average is the mean of its 2^d children. */
static double restrict_cell(int dim, int nf, const double *Af, int64_t off,
                            const int *p)
{
    int c[3] = {2 * p[0], 2 * p[1], dim == 3 ? 2 * p[2] : 0};
#define AF(dx, dy, dz) Af[off + (c[0] + (dx)) + (int64_t)nf * ((c[1] + (dy)) + (int64_t)nf * (c[2] + (dz)))]
    if (dim == 2)
        return 0.25 * ((AF(0, 0, 0) + AF(1, 0, 0)) + (AF(0, 1, 0) + AF(1, 1, 0)));
    return 0.125 * (((AF(0, 0, 0) + AF(1, 0, 0)) + (AF(0, 1, 0) + AF(1, 1, 0))) +
                    ((AF(0, 0, 1) + AF(1, 0, 1)) + (AF(0, 1, 1) + AF(1, 1, 1))));
#undef AF
}

/* Harten's third-order cell-average prediction in 1D (quadratic
 * interpolation of the parent and its two neighbours): lower child
 * q0 + (q_{-1} - q_{+1}) / 8, upper child q0 - (q_{-1} - q_{+1}) / 8. */
static double pred1(double qm, double q0, double qp, int upper)
{
    double s8 = upper ? -0.125 : 0.125;
    return q0 + s8 * (qm - qp);
}

/* Prediction of child ch (bits: x, y, z) of coarse cell p for one field of
 * array Ac (n_c^d grid), tensor product applied x, then y, then z. */
static double predict_child(int dim, int nc, int bc, const double *Ac,
                            int64_t off, const int *p, const int *ch)
{
    int xs[3], ys[3], zs[3];
    for (int k = 0; k < 3; ++k) {
        xs[k] = bcmap(p[0] + k - 1, nc, bc);
        ys[k] = bcmap(p[1] + k - 1, nc, bc);
        zs[k] = dim == 3 ? bcmap(p[2] + k - 1, nc, bc) : 0;
    }
#define AC(x, y, z) Ac[off + (x) + (int64_t)nc * ((y) + (int64_t)nc * (z))]
    if (dim == 2) {
        double r[3];
        for (int j = 0; j < 3; ++j)
            r[j] = pred1(AC(xs[0], ys[j], 0), AC(xs[1], ys[j], 0), AC(xs[2], ys[j], 0), ch[0]);
        return pred1(r[0], r[1], r[2], ch[1]);
    }
    double s[3];
    for (int k = 0; k < 3; ++k) {
        double r[3];
        for (int j = 0; j < 3; ++j)
            r[j] = pred1(AC(xs[0], ys[j], zs[k]), AC(xs[1], ys[j], zs[k]), AC(xs[2], ys[j], zs[k]), ch[0]);
        s[k] = pred1(r[0], r[1], r[2], ch[1]);
    }
    return pred1(s[0], s[1], s[2], plant == PLANT_PRED_ZSWAP ? !ch[2] : ch[2]);
#undef AC
}

/* ------------------------------------------------------------------------ */
/* standalone operators on caller arrays (used by the tests as pins)         */
/* ------------------------------------------------------------------------ */

void orc_prim2cons(int dim, double g, int64_t ncell, const double *W, double *Q)
{
    int nv = dim + 2;
    for (int64_t i = 0; i < ncell; ++i) {
        double w[NVMAX], q[NVMAX];
        for (int f = 0; f < nv; ++f) w[f] = W[f * ncell + i];
        prim2cons(dim, g, w, q);
        for (int f = 0; f < nv; ++f) Q[f * ncell + i] = q[f];
    }
}

void orc_cons2prim(int dim, double g, int64_t ncell, const double *Q, double *W)
{
    int nv = dim + 2;
    for (int64_t i = 0; i < ncell; ++i) {
        double w[NVMAX], q[NVMAX];
        for (int f = 0; f < nv; ++f) q[f] = Q[f * ncell + i];
        cons2prim(dim, g, q, w);
        for (int f = 0; f < nv; ++f) W[f * ncell + i] = w[f];
    }
}

/* AUSM+ flux of a single face; wL, wR primitive (nv values each). */
void orc_ausm_plus(int dim, double g, int dn, const double *wL, const double *wR, double *F)
{
    ausm_plus(dim, g, dn, wL, wR, F, 0);
}

void orc_ausm_plus_speed(int dim, double g, int dn, const double *wL, const double *wR, double *F, int speed)
{
    ausm_plus(dim, g, dn, wL, wR, F, speed);
}

double orc_slope(double wm, double w0, double wp) { return slope_va(wm, w0, wp); }
double orc_minmod(double wm, double w0, double wp) { return slope_minmod(wm, w0, wp); }
void orc_ausmdv(int dim, double g, int dn, const double *wL, const double *wR, double *F)
{
    ausmdv(dim, g, dn, wL, wR, F);
}
void orc_phys_flux(int dim, double g, int dn, const double *w, double *F) { phys_flux(dim, g, dn, w, F); }

/* Restrict one field-major array (nv fields) from an (2 nc)^d grid to nc^d. */
void orc_restrict(int dim, int nv, int nc, const double *Af, double *Ac)
{
    int nf = 2 * nc;
    int64_t Nc = ncells(dim, nc), Nf = ncells(dim, nf);
    for (int f = 0; f < nv; ++f)
        for (int64_t i = 0; i < Nc; ++i) {
            int p[3];
            cdecode(dim, nc, i, p);
            Ac[f * Nc + i] = restrict_cell(dim, nf, Af, f * Nf, p);
        }
}

/* Predict every child of an nc^d grid onto a (2 nc)^d grid. */
void orc_predict(int dim, int nv, int nc, int bc, const double *Ac, double *Af)
{
    int nf = 2 * nc;
    int64_t Nc = ncells(dim, nc), Nf = ncells(dim, nf);
    for (int f = 0; f < nv; ++f)
        for (int64_t i = 0; i < Nf; ++i) {
            int k[3], p[3], ch[3];
            cdecode(dim, nf, i, k);
            for (int d = 0; d < 3; ++d) { p[d] = k[d] / 2; ch[d] = k[d] & 1; }
            Af[f * Nf + i] = predict_child(dim, nc, bc, Ac, f * Nc, p, ch);
        }
}

/* ------------------------------------------------------------------------ */
/* the hierarchy                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int lvl, o[3], size[3];   /* origin and extents in cells of level lvl (2D: size[2] = 1) */
} orc_patch;

typedef struct {
    int dim, L, n0, bc, nv;
    double g, lo, hi, eps, eta;
    int pmin, pmax;
    int n[MAXL];
    double dx[MAXL];
    double *Q[MAXL];     /* current state                                 */
    double *Qs[MAXL];    /* RK2 intermediate state Q*                      */
    double *Qo[MAXL];    /* level state at the start of its step (LTS)     */
    uint8_t *act[MAXL];  /* cell belongs to a patch of its level           */
    uint8_t *nact[MAXL]; /* scratch for the new hierarchy                  */
    uint8_t *sig[MAXL];  /* significant detail (0 .. L-2)                  */
    uint8_t *flag[MAXL]; /* final refinement flags after closure (0..L-2)  */
    double *D[MAXL];     /* detail norm (0 .. L-2)                         */
    double *regC[MAXL];  /* LTS flux registers, coarse side [d][f][cell]   */
    double *regF[MAXL];  /* LTS flux registers, fine side [sub][d][f][cell] */
    orc_patch *patches;
    int npatch, cappatch;
    int no_reflux;       /* test-only planted mistake: skip the flux correction */
    int scheme;          /* 0: MR scheme (MUSCL, van Albada, AUSM+, midpoint RK2);
                            1: AMR scheme (MUSCL-Hancock, Minmod, AUSMDV) */
    int crit;            /* refinement criterion: 0 MR details (Sec. 2.1), 1 the
                            scaled-gradient indicators of the AMR method (Sec. 2.2) */
    double eps_p;        /* criterion 1: pressure threshold (<= 0: density only) */
    int eps_levels;      /* criterion 0: 1 = level-dependent thresholds (eps_at) */
    int rk;              /* MR scheme time stepping: 0 the midpoint rule, 1 Heun */
    int ausm_speed;      /* MR scheme: AUSM+ interface sound speed (ausm_plus) */
    int tiler;           /* 0 block tiler (tile_block), 1 Berger-Rigoutsos (br_block) */
    int cfl_max;         /* CFL signal speed: 0 sum_d (|v_d| + c), 1 max_d (|v_d| + c) */
} orc_h;

static int64_t hN(const orc_h *h, int l) { return ncells(h->dim, h->n[l]); }

void orc_h_free(orc_h *h)
{
    if (!h) return;
    for (int l = 0; l < h->L; ++l) {
        free(h->Q[l]); free(h->Qs[l]); free(h->Qo[l]);
        free(h->act[l]); free(h->nact[l]); free(h->sig[l]); free(h->flag[l]);
        free(h->D[l]); free(h->regC[l]); free(h->regF[l]);
    }
    free(h->patches);
    free(h);
}

/* Returns NULL on invalid parameters or allocation failure. */
orc_h *orc_h_new(int dim, int L, int n0, int bc, double g, double lo, double hi,
                 double eps, double eta, int pmin, int pmax)
{
    if ((dim != 2 && dim != 3) || L < 1 || L > MAXL || n0 < 1) return NULL;
    if (L > 1 && ((2 * n0) % pmax != 0 || pmin < 2 || pmax < pmin)) return NULL;
    orc_h *h = (orc_h *)calloc(1, sizeof(orc_h));
    if (!h) return NULL;
    h->dim = dim; h->L = L; h->n0 = n0; h->bc = bc; h->nv = dim + 2;
    h->g = g; h->lo = lo; h->hi = hi; h->eps = eps; h->eta = eta;
    h->pmin = pmin; h->pmax = pmax;
    for (int l = 0; l < L; ++l) {
        h->n[l] = n0 << l;
        h->dx[l] = (hi - lo) / (double)h->n[l];
        int64_t N = hN(h, l);
        h->Q[l] = (double *)calloc((size_t)(h->nv * N), sizeof(double));
        h->Qs[l] = (double *)calloc((size_t)(h->nv * N), sizeof(double));
        h->act[l] = (uint8_t *)malloc((size_t)N);
        h->nact[l] = (uint8_t *)malloc((size_t)N);
        if (!h->Q[l] || !h->Qs[l] || !h->act[l] || !h->nact[l]) { orc_h_free(h); return NULL; }
        memset(h->act[l], l == 0 ? 1 : 0, (size_t)N);
        if (l < L - 1) {
            h->sig[l] = (uint8_t *)calloc((size_t)N, 1);
            h->flag[l] = (uint8_t *)calloc((size_t)N, 1);
            h->D[l] = (double *)calloc((size_t)N, sizeof(double));
            if (!h->sig[l] || !h->flag[l] || !h->D[l]) { orc_h_free(h); return NULL; }
        }
    }
    return h;
}

double *orc_h_level(orc_h *h, int l) { return h->Q[l]; }
double *orc_h_level_stage(orc_h *h, int l) { return h->Qs[l]; }
uint8_t *orc_h_active(orc_h *h, int l) { return h->act[l]; }
uint8_t *orc_h_flags(orc_h *h, int l) { return l < h->L - 1 ? h->flag[l] : NULL; }
double *orc_h_details(orc_h *h, int l) { return l < h->L - 1 ? h->D[l] : NULL; }
int orc_h_n(const orc_h *h, int l) { return h->n[l]; }
double orc_h_dx(const orc_h *h, int l) { return h->dx[l]; }

/* covered: the cell's children belong to a patch of the next finer level */
static int covered(const orc_h *h, const uint8_t *const *act, int l, const int *p)
{
    if (l + 1 >= h->L) return 0;
    int c[3] = {2 * p[0], 2 * p[1], h->dim == 3 ? 2 * p[2] : 0};
    return act[l + 1][cidx(h->n[l + 1], c)];
}

static int is_leaf(const orc_h *h, int l, const int *p)
{
    return h->act[l][cidx(h->n[l], p)] && !covered(h, (const uint8_t *const *)h->act, l, p);
}

/* ghost cell: outside every patch of its level but within two cells
 * (max-norm, through the boundary map) of a cell that is inside one. */
static int is_ghost(const orc_h *h, int l, const int *p)
{
    int n = h->n[l];
    if (l == 0 || h->act[l][cidx(n, p)]) return 0;
    int r3 = h->dim == 3 ? 2 : 0;
    for (int dz = -r3; dz <= r3; ++dz)
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                int q[3] = {bcmap(p[0] + dx, n, h->bc), bcmap(p[1] + dy, n, h->bc),
                            h->dim == 3 ? bcmap(p[2] + dz, n, h->bc) : 0};
                if (h->act[l][cidx(n, q)]) return 1;
            }
    return 0;
}

/* ---- inter-level transfer on the hierarchy ---- */

/* Projection onto every covered cell, finest level first (Sec. 2.2: cells
 * covered by finer patches hold averaged fine values). */
static void h_restrict(orc_h *h, double **A)
{
    for (int l = h->L - 2; l >= 0; --l) {
        int n = h->n[l];
        int64_t N = hN(h, l), Nf = hN(h, l + 1);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            int p[3];
            cdecode(h->dim, n, i, p);
            if (!h->act[l][i] || !covered(h, (const uint8_t *const *)h->act, l, p)) continue;
            for (int f = 0; f < h->nv; ++f)
                A[l][f * N + i] = restrict_cell(h->dim, h->n[l + 1], A[l + 1], f * Nf, p);
        }
    }
}

/* Ghost cells of every level l >= 1 by prediction from level l-1
 * (Sec. 2.2: spatial interpolation at internal refinement boundaries; the
 * interpolation is the MR prediction of Sec. 2.1). */
static void h_ghost(orc_h *h, double **A)
{
    for (int l = 1; l < h->L; ++l) {
        int n = h->n[l];
        int64_t N = hN(h, l), Nc = hN(h, l - 1);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            int k[3], p[3], ch[3];
            cdecode(h->dim, n, i, k);
            if (!is_ghost(h, l, k)) continue;
            for (int d = 0; d < 3; ++d) { p[d] = k[d] / 2; ch[d] = k[d] & 1; }
            for (int f = 0; f < h->nv; ++f)
                A[l][f * N + i] = predict_child(h->dim, h->n[l - 1], h->bc, A[l - 1], f * Nc, p, ch);
        }
    }
}

/* Same as h_ghost, but the coarse data is the linear time interpolation
 * (1 - theta) A_old + theta A_new at level l-1 (Sec. 2.2, space-time
 * interpolation with recursive time steps).  Only for level l. */
static void h_ghost_time(orc_h *h, int l, double **A, double **Aold, double **Anew,
                         double theta)
{
    int n = h->n[l], nc = h->n[l - 1];
    int64_t N = hN(h, l), Nc = hN(h, l - 1);
    double *tmp = (double *)malloc((size_t)(h->nv * Nc) * sizeof(double));
    for (int64_t i = 0; i < h->nv * Nc; ++i)
        tmp[i] = (1.0 - theta) * Aold[l - 1][i] + theta * Anew[l - 1][i];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int k[3], p[3], ch[3];
        cdecode(h->dim, n, i, k);
        if (!is_ghost(h, l, k)) continue;
        for (int d = 0; d < 3; ++d) { p[d] = k[d] / 2; ch[d] = k[d] & 1; }
        for (int f = 0; f < h->nv; ++f)
            A[l][f * N + i] = predict_child(h->dim, nc, h->bc, tmp, f * Nc, p, ch);
    }
    free(tmp);
}

void orc_h_restrict(orc_h *h) { h_restrict(h, h->Q); }

/* Test-only: impose the patch membership of level l >= 1 (a fixed
 * hierarchy for runs without regrid); the caller keeps it properly nested
 * and then projects and fills the ghost cells. */
void orc_h_set_active(orc_h *h, int l, const uint8_t *mask)
{
    if (l < 1 || l >= h->L) return;
    memcpy(h->act[l], mask, (size_t)hN(h, l));
    memcpy(h->nact[l], mask, (size_t)hN(h, l));
}
void orc_h_ghost(orc_h *h) { h_ghost(h, h->Q); }

/* ---- the finite-volume update ---- */

/* Face flux of the hierarchy's scheme at the face between cell c and
 * c + e_dn of a level of n cells per side: the MR scheme's AUSM+ of the
 * MUSCL face states, or the AMR scheme's AUSMDV of the evolved Hancock face
 * values, hl = (dt / 2) / dx of that level (unused by the MR scheme). */
static void level_flux(const orc_h *h, int n, const double *A, int dn, const int *c, double hl, double *F)
{
    if (h->scheme == 1) face_flux_hancock(h->dim, n, h->bc, h->g, A, dn, c, hl, F);
    else face_flux(h->dim, n, h->bc, h->g, A, dn, c, F, h->ausm_speed);
}

/* Flux across the face between coarse cell p (level l) and its covered
 * neighbour on side s (+1 / -1) of axis dn: the mean of the 2^(d-1) level
 * l+1 fluxes along that face, computed from level l+1 data (the virtual
 * leaves of Sec. 2.1, which keep the flux balance between levels
 * conservative).  hlf: the AMR scheme's (dt / 2) / dx of level l+1. */
static void flux_fine_mean(const orc_h *h, int l, double **src, int dn,
                           const int *p, int s, double hlf, double *F)
{
    int dim = h->dim, nf = h->n[l + 1], nv = h->nv;
    int t1 = dn == 0 ? 1 : 0, t2 = dn == 2 ? 1 : 2;
    int base[3] = {2 * p[0], 2 * p[1], dim == 3 ? 2 * p[2] : 0};
    base[dn] = s > 0 ? 2 * p[dn] + 1 : 2 * p[dn] - 1;
    if (dim == 2) {
        double Fa[NVMAX], Fb[NVMAX];
        int c0[3] = {base[0], base[1], 0}, c1[3] = {base[0], base[1], 0};
        c1[t1] += 1;
        level_flux(h, nf, src[l + 1], dn, c0, hlf, Fa);
        level_flux(h, nf, src[l + 1], dn, c1, hlf, Fb);
        for (int f = 0; f < nv; ++f) F[f] = 0.5 * (Fa[f] + Fb[f]);
        return;
    }
    double F00[NVMAX], F10[NVMAX], F01[NVMAX], F11[NVMAX];
    int c00[3] = {base[0], base[1], base[2]};
    int c10[3] = {base[0], base[1], base[2]};
    int c01[3] = {base[0], base[1], base[2]};
    int c11[3] = {base[0], base[1], base[2]};
    c10[t1] += 1; c01[t2] += 1; c11[t1] += 1; c11[t2] += 1;
    level_flux(h, nf, src[l + 1], dn, c00, hlf, F00);
    level_flux(h, nf, src[l + 1], dn, c10, hlf, F10);
    level_flux(h, nf, src[l + 1], dn, c01, hlf, F01);
    level_flux(h, nf, src[l + 1], dn, c11, hlf, F11);
    for (int f = 0; f < nv; ++f) F[f] = 0.25 * ((F00[f] + F10[f]) + (F01[f] + F11[f]));
}

/* One explicit stage on every leaf of level l:
 *   out = base - lam * ((dF_1 + dF_2) + dF_3),  dF_d = F_{+1/2} - F_{-1/2},
 * the semi-discrete form dQ/dt = -F(Q) of Sec. 2 with fluxes from src.
 * A face next to a covered cell takes the fine-flux mean (flux_fine_mean).
 * dt: the step, for the AMR scheme's half-step predictor of each level.
 * blend (Heun's second stage): the base is (base + src) / 2. */
static void h_fv_level(orc_h *h, int l, double **src, double **base,
                       double **out, double lam, double dt, int blend)
{
    int dim = h->dim, n = h->n[l], nv = h->nv;
    int64_t N = hN(h, l);
    double hl = (dt * 0.5) / h->dx[l];
    double hlf = l + 1 < h->L ? (dt * 0.5) / h->dx[l + 1] : 0.0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
        int p[3];
        cdecode(dim, n, i, p);
        if (!is_leaf(h, l, p)) continue;
        double dF[3][NVMAX];
        for (int d = 0; d < dim; ++d) {
            double Fhi[NVMAX], Flo[NVMAX];
            int nb[3] = {p[0], p[1], p[2]};
            nb[d] = bcmap(p[d] + 1, n, h->bc);
            int fm = plant != PLANT_NO_FINE_MEAN;
            if (fm && covered(h, (const uint8_t *const *)h->act, l, nb))
                flux_fine_mean(h, l, src, d, p, +1, hlf, Fhi);
            else
                level_flux(h, n, src[l], d, p, hl, Fhi);
            nb[d] = bcmap(p[d] - 1, n, h->bc);
            if (fm && covered(h, (const uint8_t *const *)h->act, l, nb)) {
                flux_fine_mean(h, l, src, d, p, -1, hlf, Flo);
            } else {
                int lc[3] = {p[0], p[1], p[2]};
                lc[d] = p[d] - 1;
                level_flux(h, n, src[l], d, lc, hl, Flo);
            }
            for (int f = 0; f < nv; ++f) dF[d][f] = Fhi[f] - Flo[f];
        }
        for (int f = 0; f < nv; ++f) {
            double R = dF[0][f] + dF[1][f];
            if (dim == 3) R = R + dF[2][f];
            double b = blend ? 0.5 * (base[l][f * N + i] + src[l][f * N + i]) : base[l][f * N + i];
            out[l][f * N + i] = b - lam * R;
        }
    }
}

/* CFL time step over all leaves: dt = min over levels of cfl dx_l / S_l,
 * S_l the largest signal speed of the level's leaves, sum_d (|v_d| + c) (the
 * default) or max_d (|v_d| + c) (cfl_max), clipped to reach t_end. */
double orc_h_cfl(orc_h *h, double cfl, double t, double t_end, double *smax_out)
{
    int dim = h->dim;
    double dt = INFINITY;
    for (int l = 0; l < h->L; ++l) {
        int n = h->n[l];
        int64_t N = hN(h, l);
        double smax = 0.0;
        int any = 0;
        for (int64_t i = 0; i < N; ++i) {
            int p[3];
            cdecode(dim, n, i, p);
            if (!is_leaf(h, l, p)) continue;
            double q[NVMAX], w[NVMAX];
            for (int f = 0; f < h->nv; ++f) q[f] = h->Q[l][f * N + i];
            cons2prim(dim, h->g, q, w);
            double c = sqrt((h->g * w[dim + 1]) / w[0]);
            double S = 0.0;
            for (int d = 0; d < dim; ++d) {
                double sd = fabs(w[1 + d]) + c;
                S = h->cfl_max ? (sd > S ? sd : S) : S + sd;
            }
            if (S > smax) smax = S;
            any = 1;
        }
        if (smax_out) smax_out[l] = smax;
        if (any) {
            double dtl = (cfl * h->dx[l]) / smax;
            if (dtl < dt) dt = dtl;
        }
    }
    if (dt > t_end - t) dt = t_end - t;
    return dt;
}

/* Conserved totals sum over leaves of Q_f |cell|, with Neumaier's
 * compensated summation. */
void orc_h_totals(orc_h *h, double *tot)
{
    int dim = h->dim;
    for (int f = 0; f < h->nv; ++f) {
        double s = 0.0, comp = 0.0;
        for (int l = 0; l < h->L; ++l) {
            int n = h->n[l];
            int64_t N = hN(h, l);
            double vol = dim == 2 ? h->dx[l] * h->dx[l] : h->dx[l] * h->dx[l] * h->dx[l];
            for (int64_t i = 0; i < N; ++i) {
                int p[3];
                cdecode(dim, n, i, p);
                if (!is_leaf(h, l, p)) continue;
                double x = h->Q[l][f * N + i] * vol;
                double t = s + x;
                if (fabs(s) >= fabs(x)) comp += (s - t) + x;
                else comp += (x - t) + s;
                s = t;
            }
        }
        tot[f] = s + comp;
    }
}

void orc_h_counts(orc_h *h, int64_t *leaves, int64_t *active)
{
    for (int l = 0; l < h->L; ++l) {
        int n = h->n[l];
        int64_t N = hN(h, l), nl = 0, na = 0;
        for (int64_t i = 0; i < N; ++i) {
            int p[3];
            cdecode(h->dim, n, i, p);
            if (h->act[l][i]) ++na;
            if (is_leaf(h, l, p)) ++nl;
        }
        leaves[l] = nl;
        active[l] = na;
    }
}

/* ---- MR analysis, thresholding, closure and tiling ---- */

/* Details of every refined level-l cell: the largest magnitude of the
 * prediction error of its children's densities (Sec. 2.1: details are the
 * prediction errors between consecutive levels).  A detail is significant
 * when it is not smaller than eps (hard thresholding; the same eps on every
 * level). */
/* Refinement indicators of the AMR method (Sec. 2.2): a cell P of level l
 * (in a patch of that level) is flagged when |w(P + a) - w(P)| > eps_w for
 * one of its neighbours P + a, a in {0,1}^d other than 0, with w = rho
 * (eps_rho = eps) and w = p (eps_p, when positive).  Neighbours outside the
 * patches are ghost cells (filled first, by prediction); D receives the
 * largest density difference. */
static void h_gradient(orc_h *h)
{
    h_ghost(h, h->Q);
    int dim = h->dim, nv = h->nv;
    for (int l = 0; l < h->L - 1; ++l) {
        int n = h->n[l];
        int64_t N = hN(h, l);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            int p[3];
            cdecode(dim, n, i, p);
            h->D[l][i] = 0.0;
            h->sig[l][i] = 0;
            if (!h->act[l][i]) continue;
            double q[NVMAX], w0[NVMAX];
            for (int f = 0; f < nv; ++f) q[f] = h->Q[l][f * N + i];
            cons2prim(dim, h->g, q, w0);
            double dr = 0.0, dpm = 0.0;
            int na = 1 << dim;
            for (int a = 1; a < na; ++a) {
                int c[3] = {bcmap(p[0] + (a & 1), n, h->bc), bcmap(p[1] + ((a >> 1) & 1), n, h->bc),
                            dim == 3 ? bcmap(p[2] + ((a >> 2) & 1), n, h->bc) : 0};
                double qa[NVMAX], wa[NVMAX];
                int64_t j = cidx(n, c);
                for (int f = 0; f < nv; ++f) qa[f] = h->Q[l][f * N + j];
                cons2prim(dim, h->g, qa, wa);
                double er = fabs(wa[0] - w0[0]), ep = fabs(wa[dim + 1] - w0[dim + 1]);
                if (er > dr) dr = er;
                if (ep > dpm) dpm = ep;
            }
            h->D[l][i] = dr;
            h->sig[l][i] = dr > h->eps || (h->eps_p > 0.0 && dpm > h->eps_p);
        }
    }
}

/* Threshold of the details of level l: eps, or with level-dependent
 * thresholds eps_l = 2^(d (l + 2 - L)) eps, eps on the finest details
 * (l = L-2) and halved d times per coarser level (Harten's scaling of the
 * thresholds with the cell volume). */
static double eps_at(const orc_h *h, int l)
{
    return h->eps_levels ? ldexp(h->eps, h->dim * (l + 2 - h->L)) : h->eps;
}

static void h_details(orc_h *h)
{
    if (h->crit == 1) {
        h_gradient(h);
        return;
    }
    for (int l = 0; l < h->L - 1; ++l) {
        int n = h->n[l], nf = h->n[l + 1];
        int64_t N = hN(h, l);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            int p[3];
            cdecode(h->dim, n, i, p);
            h->D[l][i] = 0.0;
            h->sig[l][i] = 0;
            if (!h->act[l][i] || !covered(h, (const uint8_t *const *)h->act, l, p)) continue;
            double Dm = 0.0;
            int nch = 1 << h->dim;
            for (int k = 0; k < nch; ++k) {
                int ch[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
                int c[3] = {2 * p[0] + ch[0], 2 * p[1] + ch[1], h->dim == 3 ? 2 * p[2] + ch[2] : 0};
                double rho = h->Q[l + 1][cidx(nf, c)];
                double pr = predict_child(h->dim, n, h->bc, h->Q[l], 0, p, ch);
                double dd = fabs(rho - pr);
                if (dd > Dm) Dm = dd;
            }
            h->D[l][i] = Dm;
            h->sig[l][i] = Dm >= eps_at(h, l);
        }
    }
}

/* raw refinement flag of level-l cell p (l <= L-2): keep cells with
 * significant details, and refine significant cells by one more level
 * (Sec. 2.1, refinement: the mesh is refined by one level before the
 * evolution). */
static int raw_flag(const orc_h *h, int l, const int *p)
{
    int n = h->n[l];
    if (h->sig[l][cidx(n, p)]) return 1;
    if (l >= 1 && h->crit == 0) {
        int q[3] = {p[0] / 2, p[1] / 2, p[2] / 2};
        if (h->sig[l - 1][cidx(h->n[l - 1], q)]) return 1;
    }
    return 0;
}

/* Final flags of level l (decide level l+1 of the new hierarchy):
 *  1. raw flags dilated by one cell (buffer layer, Sec. 2.2; gradedness,
 *     Sec. 2.1);
 *  2. nesting: level-l+1 cells within two cells of a level-l+1 cell covered
 *     by the new level l+2 must exist, so their parents are flagged. */
static void h_flags(orc_h *h, int l)
{
    int dim = h->dim, n = h->n[l], nf = h->n[l + 1];
    int64_t N = hN(h, l);
    int r3 = dim == 3 ? 1 : 0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int p[3];
        cdecode(dim, n, i, p);
        int fl = 0;
        for (int dz = -r3; dz <= r3 && !fl; ++dz)
            for (int dy = -1; dy <= 1 && !fl; ++dy)
                for (int dx = -1; dx <= 1 && !fl; ++dx) {
                    int q[3] = {bcmap(p[0] + dx, n, h->bc), bcmap(p[1] + dy, n, h->bc),
                                dim == 3 ? bcmap(p[2] + dz, n, h->bc) : 0};
                    if (raw_flag(h, l, q)) fl = 1;
                }
        if (!fl && l + 2 < h->L) {
            /* children span 2p .. 2p+1; cells within 2 of them: 2p-2 .. 2p+3 */
            int z0 = dim == 3 ? -2 : 0, z1 = dim == 3 ? 3 : 0;
            for (int dz = z0; dz <= z1 && !fl; ++dz)
                for (int dy = -2; dy <= 3 && !fl; ++dy)
                    for (int dx = -2; dx <= 3 && !fl; ++dx) {
                        int q[3] = {bcmap(2 * p[0] + dx, nf, h->bc), bcmap(2 * p[1] + dy, nf, h->bc),
                                    dim == 3 ? bcmap(2 * p[2] + dz, nf, h->bc) : 0};
                        if (covered(h, (const uint8_t *const *)h->nact, l + 1, q)) fl = 1;
                    }
        }
        h->flag[l][i] = (uint8_t)fl;
    }
}

/* A patch of level lvl: origin o, extents S[0..2] cells (S[2] = 1 in 2D);
 * its cells join the new hierarchy. */
static void emit_patch(orc_h *h, int lvl, const int *o, const int *S)
{
    if (h->npatch == h->cappatch) {
        h->cappatch = h->cappatch ? 2 * h->cappatch : 256;
        h->patches = (orc_patch *)realloc(h->patches, (size_t)h->cappatch * sizeof(orc_patch));
    }
    orc_patch *P = &h->patches[h->npatch++];
    P->lvl = lvl;
    for (int d = 0; d < 3; ++d) {
        P->o[d] = o[d];
        P->size[d] = S[d];
    }
    int nf = h->n[lvl];
    for (int z = 0; z < S[2]; ++z)
        for (int y = 0; y < S[1]; ++y)
            for (int x = 0; x < S[0]; ++x) {
                int c[3] = {o[0] + x, o[1] + y, h->dim == 3 ? o[2] + z : 0};
                h->nact[lvl][cidx(nf, c)] = 1;
            }
}

/* Patch generation for level l+1 from the flags of level l (stands in for
 * the clustering of Sec. 2.2, same efficiency rule): an aligned block of
 * S^d level-(l+1) cells whose parents include flagged ones becomes a patch
 * when the flagged fraction reaches eta or S is the smallest patch size;
 * otherwise it is split into its 2^d half-size blocks. */
static void tile_block(orc_h *h, int l, const int *o, int S)
{
    int dim = h->dim, n = h->n[l], hs = S / 2;
    int64_t cnt = 0, cells = dim == 2 ? (int64_t)hs * hs : (int64_t)hs * hs * hs;
    int z1 = dim == 3 ? hs : 1;
    for (int z = 0; z < z1; ++z)
        for (int y = 0; y < hs; ++y)
            for (int x = 0; x < hs; ++x) {
                int c[3] = {o[0] / 2 + x, o[1] / 2 + y, dim == 3 ? o[2] / 2 + z : 0};
                cnt += h->flag[l][cidx(n, c)];
            }
    if (cnt == 0) return;
    if (S == h->pmin || (double)cnt >= h->eta * (double)cells) {
        int ext[3] = {S, S, dim == 3 ? S : 1};
        emit_patch(h, l + 1, o, ext);
        return;
    }
    int nch = 1 << dim;
    for (int k = 0; k < nch; ++k) {
        int oc[3] = {o[0] + hs * (k & 1), o[1] + hs * ((k >> 1) & 1), dim == 3 ? o[2] + hs * ((k >> 2) & 1) : 0};
        tile_block(h, l, oc, hs);
    }
}

/* Berger-Rigoutsos clustering (the AMR method's clustering, Sec. 2.2;
 * Berger and Rigoutsos 1991), a variant tiler: inside one block of pmax^d
 * level-(l+1) cells at o, on the grid of its R^d sub-blocks of pmin^d cells
 * (R = pmax / pmin; patches stay unions of whole sub-blocks), each
 * sub-block weighted by the flagged level-l cells among its parents.  A box
 * of sub-blocks (inclusive bounds lo..hi per axis) is
 *   1. shrunk to the sub-blocks with flagged cells (nothing left: dropped);
 *   2. emitted when its flagged fraction of parent cells reaches eta, or it
 *      is a single sub-block;
 *   3. otherwise cut at a hole: a zero of the signature (flagged cells per
 *      slice) along an axis, the axes taken longest first (ties: x, y, z),
 *      the hole nearest the middle (ties: the lower one), the cut just
 *      above it;
 *   4. else at the strongest inflection of the signature: between slices k
 *      and k+1 where the second differences D[i] = s[i-1] - 2 s[i] + s[i+1]
 *      change sign, strength |D[k] - D[k+1]|, the strongest over all axes
 *      (ties: axis order of step 3, then nearest the middle, then lower k);
 *   5. else halved along its longest axis (ties: x, y, z), the lower half
 *      taking the smaller share;
 *   and the two parts are clustered in turn, the lower one first. */
/* Boxes found so far: inclusive sub-block bounds lo[3], hi[3] each. */
typedef struct {
    int n, lo[512][3], hi[512][3];
} br_out;

static void br_box(int dim, int q, double eta, const int W[8][8][8], const int *lo0, const int *hi0, br_out *out)
{
    int lo[3], hi[3];
    /* 1. shrink */
    int any = 0;
    for (int d = 0; d < 3; ++d) { lo[d] = hi0[d] + 1; hi[d] = lo0[d] - 1; }
    for (int z = lo0[2]; z <= hi0[2]; ++z)
        for (int y = lo0[1]; y <= hi0[1]; ++y)
            for (int x = lo0[0]; x <= hi0[0]; ++x)
                if (W[z][y][x] > 0) {
                    int c[3] = {x, y, z};
                    for (int d = 0; d < 3; ++d) {
                        if (c[d] < lo[d]) lo[d] = c[d];
                        if (c[d] > hi[d]) hi[d] = c[d];
                    }
                    any = 1;
                }
    if (!any) return;
    /* 2. efficiency: flagged parent cells over the box's parent cells */
    int64_t flagged = 0;
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) flagged += W[z][y][x];
    int64_t cells = 1;
    for (int d = 0; d < dim; ++d) cells *= (int64_t)(hi[d] - lo[d] + 1) * q;
    int single = lo[0] == hi[0] && lo[1] == hi[1] && lo[2] == hi[2];
    if (single || (double)flagged >= eta * (double)cells) {
        for (int d = 0; d < 3; ++d) {
            out->lo[out->n][d] = lo[d];
            out->hi[out->n][d] = hi[d];
        }
        out->n++;
        return;
    }
    /* signatures */
    int sig[3][8];
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < 8; ++i) sig[d][i] = 0;
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                sig[0][x] += W[z][y][x];
                sig[1][y] += W[z][y][x];
                sig[2][z] += W[z][y][x];
            }
    /* axes, longest first (ties: lower axis) */
    int ax[3] = {0, 1, 2}, na = dim;
    for (int i = 0; i < na; ++i)
        for (int j = i + 1; j < na; ++j) {
            int li = hi[ax[i]] - lo[ax[i]], lj = hi[ax[j]] - lo[ax[j]];
            if (lj > li || (lj == li && ax[j] < ax[i])) { int t = ax[i]; ax[i] = ax[j]; ax[j] = t; }
        }
    int cut_axis = -1, cut_at = 0;   /* halves [lo, cut_at] and [cut_at + 1, hi] */
    /* 3. holes */
    for (int k = 0; k < na && cut_axis < 0; ++k) {
        int a = ax[k], best = -1, bd = 0;
        for (int i = lo[a] + 1; i <= hi[a] - 1; ++i)
            if (sig[a][i] == 0) {
                int dd = abs(2 * i - (lo[a] + hi[a]));
                if (best < 0 || dd < bd) { best = i; bd = dd; }
            }
        if (best >= 0) { cut_axis = a; cut_at = best; }
    }
    /* 4. inflections */
    if (cut_axis < 0) {
        int bs = 0, bdist = 0;
        for (int k = 0; k < na; ++k) {
            int a = ax[k];
            for (int i = lo[a] + 1; i + 1 <= hi[a] - 1; ++i) {
                int d0 = sig[a][i - 1] - 2 * sig[a][i] + sig[a][i + 1];
                int d1 = sig[a][i] - 2 * sig[a][i + 1] + sig[a][i + 2];
                if (!((d0 < 0 && d1 > 0) || (d0 > 0 && d1 < 0))) continue;
                int st = abs(d0 - d1), dist = abs(2 * i + 1 - (lo[a] + hi[a]));
                if (cut_axis < 0 || st > bs || (st == bs && a == cut_axis && dist < bdist)) {
                    cut_axis = a; cut_at = i; bs = st; bdist = dist;
                }
            }
        }
    }
    /* 5. bisection of the longest axis */
    if (cut_axis < 0) {
        cut_axis = ax[0];
        cut_at = lo[cut_axis] + (hi[cut_axis] - lo[cut_axis] + 1) / 2 - 1;
    }
    int h1[3] = {hi[0], hi[1], hi[2]}, l2[3] = {lo[0], lo[1], lo[2]};
    h1[cut_axis] = cut_at;
    l2[cut_axis] = cut_at + 1;
    br_box(dim, q, eta, W, lo, h1, out);
    br_box(dim, q, eta, W, l2, hi, out);
}

/* Clustering of an R^d grid of sub-block weights W (flagged parent cells,
 * q^d parent cells per sub-block; index [z][y][x], R <= 8): the boxes in
 * the order found, as rows {lo_x, lo_y, lo_z, hi_x, hi_y, hi_z}.  Returns
 * their number. */
int orc_br_cluster(int dim, int R, int q, double eta, const int32_t *W, int32_t *boxes)
{
    int G[8][8][8];
    memset(G, 0, sizeof(G));
    for (int z = 0; z < (dim == 3 ? R : 1); ++z)
        for (int y = 0; y < R; ++y)
            for (int x = 0; x < R; ++x) G[z][y][x] = W[x + R * (y + R * z)];
    br_out *out = (br_out *)calloc(1, sizeof(br_out));
    int lo[3] = {0, 0, 0}, hi[3] = {R - 1, R - 1, dim == 3 ? R - 1 : 0};
    br_box(dim, q, eta, (const int (*)[8][8])G, lo, hi, out);
    int n = out->n;
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            boxes[6 * i + d] = out->lo[i][d];
            boxes[6 * i + 3 + d] = out->hi[i][d];
        }
    free(out);
    return n;
}

/* One pmax block at o: the weights of its sub-blocks from the level-l flags,
 * clustered, each box a patch of level l+1. */
static void br_block(orc_h *h, int l, const int *o)
{
    int dim = h->dim, R = h->pmax / h->pmin, q = h->pmin / 2, n = h->n[l];
    int32_t W[512];
    int32_t boxes[6 * 512];
    for (int sz = 0; sz < (dim == 3 ? R : 1); ++sz)
        for (int sy = 0; sy < R; ++sy)
            for (int sx = 0; sx < R; ++sx) {
                int w = 0;
                for (int z = 0; z < (dim == 3 ? q : 1); ++z)
                    for (int y = 0; y < q; ++y)
                        for (int x = 0; x < q; ++x) {
                            int c[3] = {o[0] / 2 + sx * q + x, o[1] / 2 + sy * q + y,
                                        dim == 3 ? o[2] / 2 + sz * q + z : 0};
                            w += h->flag[l][cidx(n, c)];
                        }
                W[sx + R * (sy + R * sz)] = w;
            }
    int nb = orc_br_cluster(dim, R, q, h->eta, W, boxes);
    for (int i = 0; i < nb; ++i) {
        int oo[3], ext[3];
        for (int d = 0; d < 3; ++d) {
            oo[d] = d < dim ? o[d] + boxes[6 * i + d] * h->pmin : 0;
            ext[d] = d < dim ? (boxes[6 * i + 3 + d] - boxes[6 * i + d] + 1) * h->pmin : 1;
        }
        emit_patch(h, l + 1, oo, ext);
    }
}

/* Tile level l's flags into patches of level l+1; blocks of size pmax are
 * visited in Morton (Z) order of their block coordinates. */
static void h_tile(orc_h *h, int l)
{
    int dim = h->dim, nb = h->n[l + 1] / h->pmax;
    int64_t nbt = dim == 2 ? (int64_t)nb * nb : (int64_t)nb * nb * nb;
    memset(h->nact[l + 1], 0, (size_t)hN(h, l + 1));
    /* Morton codes range over the next power of two of nb per axis */
    int bits = 0;
    while ((1 << bits) < nb) ++bits;
    int64_t ncode = (int64_t)1 << (bits * dim);
    int64_t seen = 0;
    for (int64_t m = 0; m < ncode && seen < nbt; ++m) {
        int b[3] = {0, 0, 0};
        for (int k = 0; k < bits; ++k)
            for (int d = 0; d < dim; ++d)
                b[d] |= (int)((m >> (k * dim + d)) & 1) << k;
        if (b[0] >= nb || b[1] >= nb || b[2] >= nb) continue;
        ++seen;
        int o[3] = {b[0] * h->pmax, b[1] * h->pmax, b[2] * h->pmax};
        if (h->tiler == 1) br_block(h, l, o);
        else tile_block(h, l, o, h->pmax);
    }
}

/* Build the new hierarchy (flags, closure and tiling from the finest level
 * down, Sec. 2.2 Remesh), then predict newly created cells from the next
 * coarser level (coarse to fine) and keep the data of cells that stay. */
static void h_regrid(orc_h *h, int prolong)
{
    h->npatch = 0;
    h_details(h);
    memset(h->nact[0], 1, (size_t)hN(h, 0));
    for (int l = h->L - 2; l >= 0; --l) {
        h_flags(h, l);
        h_tile(h, l);
    }
    /* patches were emitted finest level first; order them by level */
    if (h->npatch > 1) {
        orc_patch *tmp = (orc_patch *)malloc((size_t)h->npatch * sizeof(orc_patch));
        int k = 0;
        for (int lv = 1; lv < h->L; ++lv)
            for (int i = 0; i < h->npatch; ++i)
                if (h->patches[i].lvl == lv) tmp[k++] = h->patches[i];
        memcpy(h->patches, tmp, (size_t)h->npatch * sizeof(orc_patch));
        free(tmp);
    }
    if (prolong) {
        for (int l = 1; l < h->L; ++l) {
            int n = h->n[l];
            int64_t N = hN(h, l), Nc = hN(h, l - 1);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) {
                if (!h->nact[l][i] || h->act[l][i]) continue;
                int k[3], p[3], ch[3];
                cdecode(h->dim, n, i, k);
                for (int d = 0; d < 3; ++d) { p[d] = k[d] / 2; ch[d] = k[d] & 1; }
                for (int f = 0; f < h->nv; ++f)
                    h->Q[l][f * N + i] = predict_child(h->dim, h->n[l - 1], h->bc, h->Q[l - 1], f * Nc, p, ch);
            }
            /* level l+1 predicts from level l with the new activity of l */
            memcpy(h->act[l], h->nact[l], (size_t)N);
        }
    } else {
        for (int l = 1; l < h->L; ++l) memcpy(h->act[l], h->nact[l], (size_t)hN(h, l));
    }
}

/* Initialise the hierarchy from the finest-level data already written into
 * level L-1: restrict it down through every level, analyse every level with
 * all cells present, flag, close and tile; every patch keeps the restricted
 * initial data; then fill ghost cells. */
void orc_h_init(orc_h *h)
{
    for (int l = h->L - 2; l >= 0; --l) orc_restrict(h->dim, h->nv, h->n[l], h->Q[l + 1], h->Q[l]);
    for (int l = 0; l < h->L; ++l) memset(h->act[l], 1, (size_t)hN(h, l));
    if (h->L > 1) h_regrid(h, 0);
    h_ghost(h, h->Q);
}

/* MR analysis + thresholding + closure + tiling + prediction of new cells
 * + ghost fill: the coarsening / refinement half of the MR cycle. */
void orc_h_regrid(orc_h *h)
{
    if (h->L > 1) h_regrid(h, 1);
    h_ghost(h, h->Q);
}

void orc_h_analyse(orc_h *h) { h_details(h); }

/* Replace the detail threshold (same on every level) for later analyses. */
void orc_h_set_eps(orc_h *h, double eps) { h->eps = eps; }
void orc_h_set_eps_levels(orc_h *h, int on) { h->eps_levels = on != 0; }

int orc_h_npatch(const orc_h *h) { return h->npatch; }

/* Test-only: plant the mistake of skipping the flux correction. */
void orc_h_set_no_reflux(orc_h *h, int on) { h->no_reflux = on; }

/* patches as int32 rows {level, ox, oy, oz, sx, sy, sz} (2D: oz = 0, sz = 1) */
void orc_h_patches(const orc_h *h, int32_t *out)
{
    for (int i = 0; i < h->npatch; ++i) {
        out[7 * i + 0] = h->patches[i].lvl;
        for (int d = 0; d < 3; ++d) {
            out[7 * i + 1 + d] = h->patches[i].o[d];
            out[7 * i + 4 + d] = h->patches[i].size[d];
        }
    }
}

/* CFL signal speed: 0 the sum over axes of |v_d| + c, 1 the largest of them.
 * Returns 0, or -1. */
int orc_h_set_cfl_mode(orc_h *h, int mode)
{
    if (mode != 0 && mode != 1) return -1;
    h->cfl_max = mode;
    return 0;
}

/* Tiler: 0 the efficiency-rule block tiler (tile_block), 1 Berger-Rigoutsos
 * clustering (br_block; pmax / pmin <= 8).  Returns 0, or -1. */
int orc_h_set_tiler(orc_h *h, int tiler)
{
    if (tiler != 0 && tiler != 1) return -1;
    if (tiler == 1 && h->pmax / h->pmin > 8) return -1;
    h->tiler = tiler;
    return 0;
}

/* One explicit stage on every level (FV on leaves, projection onto covered
 * cells).  Ghost cells are filled separately. */
static void h_stage(orc_h *h, double **src, double **out, double dt, double fac, int blend)
{
    for (int l = 0; l < h->L; ++l) {
        double lam = (dt * fac) / h->dx[l];
        h_fv_level(h, l, src, h->Q, out, lam, dt, blend);
    }
    h_restrict(h, out);
}

/* The two stages of the MR scheme's RK2 step (Sec. 2), each followed by the
 * projection and the ghost fill:
 *   midpoint rule: Q* = Q - (dt/2) F(Q),  Q <- Q - dt F(Q*);
 *   Heun (a variant): Q* = Q - dt F(Q),  Q <- (Q + Q*)/2 - (dt/2) F(Q*). */
static void rk_stage1(orc_h *h, double dt)
{
    h_stage(h, h->Q, h->Qs, dt, h->rk ? 1.0 : 0.5, 0);
    h_ghost(h, h->Qs);
}

static void rk_stage2(orc_h *h, double dt)
{
    h_stage(h, h->Qs, h->Q, dt, h->rk ? 0.5 : 1.0, h->rk);
}

void orc_h_stage(orc_h *h, int stage, double dt)
{
    if (stage == 1) {
        rk_stage1(h, dt);
    } else {
        rk_stage2(h, dt);
        h_ghost(h, h->Q);
    }
}

/* Variants of the MR scheme: time stepping rk (0 midpoint, 1 Heun) and the
 * AUSM+ interface sound speed (0 mean, 1 critical).  Returns 0, or -1 for
 * an unknown value. */
int orc_h_set_variants(orc_h *h, int rk, int ausm_speed)
{
    if ((rk != 0 && rk != 1) || (ausm_speed != 0 && ausm_speed != 1)) return -1;
    h->rk = rk;
    h->ausm_speed = ausm_speed;
    return 0;
}

/* One step of the AMR scheme (Sec. 2: MUSCL-Hancock, a single corrector
 * stage) on the leaves of every level:
 *   Q^{n+1} = Q^n - (dt/dx) ((dF_1 + dF_2) + dF_3)
 * with the AUSMDV fluxes of the evolved face values, a face next to a
 * covered cell taking the mean of the finer level's fluxes; computed into
 * the stage arrays, the leaves copied back, then projected onto the covered
 * cells.
 * Ghost cells are left for the caller to fill. */
static void h_hancock(orc_h *h, double dt)
{
    for (int l = 0; l < h->L; ++l)
        h_fv_level(h, l, h->Q, h->Q, h->Qs, dt / h->dx[l], dt, 0);
    for (int l = 0; l < h->L; ++l) {
        int64_t N = hN(h, l);
        for (int64_t i = 0; i < N; ++i)
            if (h->act[l][i]) {
                int p[3];
                cdecode(h->dim, h->n[l], i, p);
                if (!is_leaf(h, l, p)) continue;
                for (int f = 0; f < h->nv; ++f) h->Q[l][f * N + i] = h->Qs[l][f * N + i];
            }
    }
    h_restrict(h, h->Q);
}

/* Select the refinement criterion: 0 the MR details (Sec. 2.1), 1 the
 * scaled-gradient indicators of the AMR method (Sec. 2.2) with the density
 * threshold eps of the hierarchy and pressure threshold eps_p (<= 0: none).
 * Returns 0, or -1 for an unknown criterion. */
int orc_h_set_criterion(orc_h *h, int crit, double eps_p)
{
    if (crit != 0 && crit != 1) return -1;
    h->crit = crit;
    h->eps_p = eps_p;
    return 0;
}

/* Select the finite-volume scheme: 0 the MR scheme, 1 the AMR scheme.
 * Returns 0, or -1 for an unknown scheme. */
int orc_h_set_scheme(orc_h *h, int scheme)
{
    if (scheme != 0 && scheme != 1) return -1;
    h->scheme = scheme;
    return 0;
}

/* One global time step (Sec. 2: explicit second-order midpoint rule):
 *   Q* = Q^n - (dt/2) F(Q^n),   Q^{n+1} = Q^n - dt F(Q*),
 * on the leaves of every level, then the MR coarsening / refinement.
 * The AMR scheme takes its single Hancock step instead, then fills the
 * ghost cells (the refinement analysis reads them) before the regrid.
 * Returns dt.  When regrid is 0 the hierarchy is left as it is. */
double orc_h_step(orc_h *h, double cfl, double t, double t_end, int regrid)
{
    double dt = orc_h_cfl(h, cfl, t, t_end, NULL);
    if (h->scheme == 1) {
        h_hancock(h, dt);
        h_ghost(h, h->Q);
        if (regrid && h->L > 1) {
            h_regrid(h, 1);
            h_ghost(h, h->Q);
        }
        return dt;
    }
    rk_stage1(h, dt);
    rk_stage2(h, dt);
    if (regrid && h->L > 1) h_regrid(h, 1);
    h_ghost(h, h->Q);
    return dt;
}

/* One step with a caller-given dt, no regrid (tests). */
void orc_h_step_fixed(orc_h *h, double dt)
{
    if (h->scheme == 1) {
        h_hancock(h, dt);
        h_ghost(h, h->Q);
        return;
    }
    rk_stage1(h, dt);
    rk_stage2(h, dt);
    h_ghost(h, h->Q);
}

/* ------------------------------------------------------------------------ */
/* local time stepping: the recursive level cycle of Sec. 2.2 (Fig. 2)      */
/* ------------------------------------------------------------------------ */

static int lts_alloc(orc_h *h)
{
    for (int l = 0; l < h->L; ++l) {
        int64_t N = hN(h, l);
        if (!h->Qo[l]) h->Qo[l] = (double *)calloc((size_t)(h->nv * N), sizeof(double));
        if (l < h->L - 1 && !h->regC[l])
            h->regC[l] = (double *)calloc((size_t)(h->dim * h->nv * N), sizeof(double));
        if (l >= 1 && !h->regF[l])
            h->regF[l] = (double *)calloc((size_t)(2 * h->dim * h->nv * N), sizeof(double));
        if (!h->Qo[l] || (l < h->L - 1 && !h->regC[l]) || (l >= 1 && !h->regF[l])) return -1;
    }
    return 0;
}

/* One explicit stage on every cell in a patch of level l (leaves and covered
 * cells, as the single-level update of Sec. 2.2 acts on whole patches),
 * with the level's own fluxes: out = Q - lam ((dF_1 + dF_2) + dF_3).  When
 * record is set (second stage), the fluxes across refinement boundaries are
 * kept for the flux correction: coarse side (a leaf next to a covered cell)
 * in regC[l], fine side (a cell next to a ghost cell) in regF[l] for
 * substep sub. */
static void h_fv_level_all(orc_h *h, int l, double **src, double **out, double lam,
                           double hl, int record, int sub)
{
    int dim = h->dim, n = h->n[l], nv = h->nv;
    int64_t N = hN(h, l);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
        if (!h->act[l][i]) continue;
        int p[3];
        cdecode(dim, n, i, p);
        int leaf = !covered(h, (const uint8_t *const *)h->act, l, p);
        double dF[3][NVMAX];
        for (int d = 0; d < dim; ++d) {
            double Fhi[NVMAX], Flo[NVMAX];
            int lc[3] = {p[0], p[1], p[2]};
            lc[d] = p[d] - 1;
            level_flux(h, n, src[l], d, p, hl, Fhi);
            level_flux(h, n, src[l], d, lc, hl, Flo);
            if (record) {
                int nh[3] = {p[0], p[1], p[2]}, nl[3] = {p[0], p[1], p[2]};
                nh[d] = bcmap(p[d] + 1, n, h->bc);
                nl[d] = bcmap(p[d] - 1, n, h->bc);
                int64_t ih = cidx(n, nh), il = cidx(n, nl);
                if (leaf && covered(h, (const uint8_t *const *)h->act, l, nh))
                    for (int f = 0; f < nv; ++f) h->regC[l][((int64_t)d * nv + f) * N + i] = Fhi[f];
                if (leaf && covered(h, (const uint8_t *const *)h->act, l, nl))
                    for (int f = 0; f < nv; ++f) h->regC[l][((int64_t)d * nv + f) * N + il] = Flo[f];
                if (l >= 1 && !h->act[l][ih])
                    for (int f = 0; f < nv; ++f)
                        h->regF[l][(((int64_t)sub * dim + d) * nv + f) * N + i] = Fhi[f];
                if (l >= 1 && !h->act[l][il])
                    for (int f = 0; f < nv; ++f)
                        h->regF[l][(((int64_t)sub * dim + d) * nv + f) * N + il] = Flo[f];
            }
            for (int f = 0; f < nv; ++f) dF[d][f] = Fhi[f] - Flo[f];
        }
        for (int f = 0; f < nv; ++f) {
            double R = dF[0][f] + dF[1][f];
            if (dim == 3) R = R + dF[2][f];
            out[l][f * N + i] = h->Q[l][f * N + i] - lam * R;
        }
    }
}

/* Projection of level l+1 onto the covered cells of level l only. */
static void h_restrict_level(orc_h *h, double **A, int l)
{
    int n = h->n[l];
    int64_t N = hN(h, l), Nf = hN(h, l + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int p[3];
        cdecode(h->dim, n, i, p);
        if (!h->act[l][i] || !covered(h, (const uint8_t *const *)h->act, l, p)) continue;
        for (int f = 0; f < h->nv; ++f)
            A[l][f * N + i] = restrict_cell(h->dim, h->n[l + 1], A[l + 1], f * Nf, p);
    }
}

/* Flux correction of level l (Sec. 2.2; Berger and Colella): at every face
 * between a leaf of level l and a covered cell, the coarse flux of the step
 * is replaced by the time and area mean of the fine fluxes of the two
 * substeps of level l+1:  Q += s lam (F_c - Fbar), s = +1 on the high face,
 * -1 on the low face, Fbar = (A_0 + A_1) / 2 with A_k the area mean of
 * substep k.  Faces are visited axis by axis, low face first. */
static void h_reflux(orc_h *h, int l, double lam)
{
    int dim = h->dim, n = h->n[l], nf = h->n[l + 1], nv = h->nv;
    int64_t N = hN(h, l), Nf = hN(h, l + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int p[3];
        cdecode(dim, n, i, p);
        if (!is_leaf(h, l, p)) continue;
        for (int d = 0; d < dim; ++d) {
            int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            for (int s = -1; s <= 1; s += 2) {
                int nb[3] = {p[0], p[1], p[2]};
                nb[d] = bcmap(p[d] + s, n, h->bc);
                if (!covered(h, (const uint8_t *const *)h->act, l, nb)) continue;
                int64_t ic = s > 0 ? i : cidx(n, nb);
                int fb[3] = {2 * p[0], 2 * p[1], dim == 3 ? 2 * p[2] : 0};
                fb[d] = bcmap(s > 0 ? 2 * p[d] + 1 : 2 * p[d] - 1, nf, h->bc);
                for (int f = 0; f < nv; ++f) {
                    double A[2];
                    for (int k = 0; k < 2; ++k) {
                        const double *R = h->regF[l + 1] + (((int64_t)k * dim + d) * nv + f) * Nf;
                        if (dim == 2) {
                            int c1[3] = {fb[0], fb[1], 0};
                            c1[t1] += 1;
                            A[k] = 0.5 * (R[cidx(nf, fb)] + R[cidx(nf, c1)]);
                        } else {
                            int c10[3] = {fb[0], fb[1], fb[2]}, c01[3] = {fb[0], fb[1], fb[2]},
                                c11[3] = {fb[0], fb[1], fb[2]};
                            c10[t1] += 1; c01[t2] += 1; c11[t1] += 1; c11[t2] += 1;
                            A[k] = 0.25 * ((R[cidx(nf, fb)] + R[cidx(nf, c10)]) +
                                           (R[cidx(nf, c01)] + R[cidx(nf, c11)]));
                        }
                    }
                    double Fbar = 0.5 * (A[0] + A[1]);
                    double Fc = h->regC[l][((int64_t)d * nv + f) * N + ic];
                    if (s > 0) h->Q[l][f * N + i] = h->Q[l][f * N + i] + lam * (Fc - Fbar);
                    else h->Q[l][f * N + i] = h->Q[l][f * N + i] - lam * (Fc - Fbar);
                }
            }
        }
    }
}

/* Advance level l by one step of dt_l (substep k of its parent's step):
 * keep the level's state at the start of the step (for the time
 * interpolation of finer ghost cells), two explicit stages on every cell of
 * the level, with second-stage ghost cells interpolated at the stage time
 * (the AMR scheme: its single Hancock step), then two substeps of level l+1
 * with ghost cells interpolated in time, the projection of level l+1 onto
 * level l and the flux correction with the fluxes of the updating stage. */
static void lts_advance(orc_h *h, int l, double dt, int k)
{
    int64_t N = hN(h, l);
    memcpy(h->Qo[l], h->Q[l], (size_t)(h->nv * N) * sizeof(double));
    /* stage times of substep k of level l within its parent's step: the
     * start, k / 2, and the midpoint, (2k + 1) / 4, as fractions of it */
    const int flat = plant == PLANT_LTS_THETA;
    if (h->scheme == 1) {
        /* the AMR scheme: one Hancock step of every cell of the level into
         * the stage array (its fluxes recorded), copied back */
        h_fv_level_all(h, l, h->Q, h->Qs, dt / h->dx[l], (dt * 0.5) / h->dx[l], 1, k);
        for (int64_t i = 0; i < N; ++i)
            if (h->act[l][i])
                for (int f = 0; f < h->nv; ++f) h->Q[l][f * N + i] = h->Qs[l][f * N + i];
    } else {
        h_fv_level_all(h, l, h->Q, h->Qs, (dt * 0.5) / h->dx[l], 0.0, 0, k);
        if (l >= 1) h_ghost_time(h, l, h->Qs, h->Qo, h->Q, flat ? 0.0 : (double)(2 * k + 1) * 0.25);
        h_fv_level_all(h, l, h->Qs, h->Q, dt / h->dx[l], 0.0, 1, k);
    }
    if (l + 1 < h->L) {
        for (int kk = 0; kk < 2; ++kk) {
            h_ghost_time(h, l + 1, h->Q, h->Qo, h->Q, flat ? 0.0 : (double)kk * 0.5);
            lts_advance(h, l + 1, dt * 0.5, kk);
        }
        h_restrict_level(h, h->Q, l);
        if (!h->no_reflux) h_reflux(h, l, dt / h->dx[l]);
    }
}

/* One level-0 step with local time steps dt_l = dt_0 / 2^l (Sec. 2.1,
 * MRLT; Sec. 2.2, AMRLT): dt_0 = min over levels of (cfl dx_l / smax_l) 2^l
 * from the leaves, clipped to reach t_end; then the MR coarsening /
 * refinement when regrid is set and a spatial ghost fill.  Returns dt_0;
 * *leaf_updates receives sum over levels of leaves_l 2^l.  -1: out of
 * memory; -2: Heun time stepping selected (the cycle uses the midpoint
 * rule). */
double orc_h_step_lts(orc_h *h, double cfl, double t, double t_end, int regrid,
                      int64_t *leaf_updates)
{
    if (h->rk != 0) return -2.0;   /* the recursive cycle steps with the midpoint rule */
    if (lts_alloc(h)) return -1.0;
    double smax[MAXL];
    orc_h_cfl(h, cfl, t, t_end, smax);
    int64_t leaves[MAXL], active[MAXL];
    orc_h_counts(h, leaves, active);
    double dt = INFINITY;
    int64_t upd = 0;
    for (int l = 0; l < h->L; ++l) {
        if (leaves[l] > 0) {
            double d = ((cfl * h->dx[l]) / smax[l]) * (double)(1 << l);
            if (d < dt) dt = d;
        }
        upd += leaves[l] << l;
    }
    if (dt > t_end - t) dt = t_end - t;
    if (leaf_updates) *leaf_updates = upd;
    lts_advance(h, 0, dt, 0);
    if (regrid && h->L > 1) h_regrid(h, 1);
    h_ghost(h, h->Q);
    return dt;
}

/* ------------------------------------------------------------------------ */
/* initial data on the finest level (cell-centre sampling)                  */
/* ------------------------------------------------------------------------ */

/* 2D four-quadrant Riemann problem (Sec. 4.1, Table 1 layout): quadrant I
 * x>x0,y>y0; II x<x0,y>y0; III x<x0,y<y0; IV x>x0,y<y0.  prim[4][4] holds
 * (rho, v1, v2, p) per quadrant I..IV. */
void orc_init_quadrant(int n, double lo, double hi, double g, double x0, double y0,
                       const double *prim, double *Q)
{
    double dx = (hi - lo) / (double)n;
    int64_t N = (int64_t)n * n;
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            double xc = lo + ((double)x + 0.5) * dx, yc = lo + ((double)y + 0.5) * dx;
            int qd;
            if (xc > x0) qd = yc > y0 ? 0 : 3;
            else qd = yc > y0 ? 1 : 2;
            double q[4];
            prim2cons(2, g, prim + 4 * qd, q);
            for (int f = 0; f < 4; ++f) Q[f * N + x + (int64_t)n * y] = q[f];
        }
}

/* 3D ellipsoid (Sec. 4.2): rotated coordinates
 *   x1r = x cos(th) - y sin(th), s = x sin(th) + y cos(th),
 *   x2r = s cos(ph) - z sin(ph), x3r = s sin(ph) + z cos(ph),
 * r^2 = (x1r/a)^2 + (x2r/b)^2 + (x3r/c)^2; inside iff r^2 < rc^2.
 * e[11] = {a, b, c, cos th, sin th, cos ph, sin ph, rc, 0, 0, 0};
 * st[4] = {rho_in, p_in, rho_out, p_out}; velocity zero. */
void orc_init_ellipsoid(int n, double lo, double hi, double g, const double *e,
                        const double *st, double *Q)
{
    double dx = (hi - lo) / (double)n;
    int64_t N = (int64_t)n * n * n;
    double rc2 = e[7] * e[7];
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                double xc = lo + ((double)x + 0.5) * dx;
                double yc = lo + ((double)y + 0.5) * dx;
                double zc = lo + ((double)z + 0.5) * dx;
                double x1 = xc * e[3] - yc * e[4];
                double s = xc * e[4] + yc * e[3];
                double x2 = s * e[5] - zc * e[6];
                double x3 = s * e[6] + zc * e[5];
                double r2 = ((x1 / e[0]) * (x1 / e[0]) + (x2 / e[1]) * (x2 / e[1])) + (x3 / e[2]) * (x3 / e[2]);
                int in = r2 < rc2;
                double w[5] = {in ? st[0] : st[2], 0.0, 0.0, 0.0, in ? st[1] : st[3]};
                double q[5];
                prim2cons(3, g, w, q);
                int64_t id = x + (int64_t)n * (y + (int64_t)n * z);
                for (int f = 0; f < 5; ++f) Q[f * N + id] = q[f];
            }
}

/* 1D Riemann problem along axis ax: left state for x_ax < x0, right state
 * otherwise; lr[6] = {rho_L, u_L, p_L, rho_R, u_R, p_R}, u along ax. */
void orc_init_riemann1d(int dim, int n, double lo, double hi, double g, int ax,
                        double x0, const double *lr, double *Q)
{
    double dx = (hi - lo) / (double)n;
    int64_t N = ncells(dim, n);
    int nv = dim + 2;
    for (int64_t i = 0; i < N; ++i) {
        int c[3];
        cdecode(dim, n, i, c);
        double xc = lo + ((double)c[ax] + 0.5) * dx;
        const double *s = xc < x0 ? lr : lr + 3;
        double w[5] = {s[0], 0.0, 0.0, 0.0, 0.0}, q[5];
        w[1 + ax] = s[1];
        w[dim + 1] = s[2];
        prim2cons(dim, g, w, q);
        for (int f = 0; f < nv; ++f) Q[f * N + i] = q[f];
    }
}
