/*
 * Plain FP64 CPU oracle for the eta-based, well-balanced central-upwind
 * (CDKLM) scheme of Brodtkorb & Holm (arXiv 1912.02457).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP implementation.
 *
 * Structure (one routine per step of the method, in the paper's order):
 *   ghost cells / boundary conditions  -- sections "Global wall boundary
 *       conditions" (eq. tradWallBCx, KxWallBCReq) and "Nesting the model"
 *   cell quantities h, h*, u, v and the Coriolis terms -- eq. desing_ours and
 *       section "Coriolis force" (north-vector projection)
 *   limited slopes of K and L -- eq. Kbackwards (and its y-analogue)
 *   face values -- eq. hE (and its W/N/S analogues), wet-dry slope fix
 *       eq. KxE_adjust, land mask section "Moving wet-dry boundary and land mask"
 *   central-upwind flux -- eq. numerical_flux
 *   right-hand side M -- eq. sw_semidiscrete with the sources of eq. swe
 *   SSP-RK2 with semi-implicit bed friction -- eq. rk2_semiimp
 *   flow relaxation nesting -- eq. frs
 *   CFL time step -- eq. cfl
 * Everything is float64, plain loops, no blocking or fusion; OpenMP only
 * distributes independent rows.
 */
#include "swe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 2 /* ghost layers: a face value needs the slope, which needs a neighbour */

/* threads of the parallel loops over rows (timing of the oracle only; the
 * rows are independent, so the result does not depend on it) */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* elementary definitions                                                    */
/* ------------------------------------------------------------------------- */

/* eq. desing_ours: h* = sign(h) max(|h|, min(h^2/(2 kappa) + kappa/2, kappa)),
 * with sign(0) = +1 so that h*(0) = kappa/2 */
double or_desing(double h, double kappa)
{
    double a = fabs(h);
    double lo = fmin(h * h / (2.0 * kappa) + 0.5 * kappa, kappa);
    double m = fmax(a, lo);
    return h < 0.0 ? -m : m;
}

/* minmod of three arguments: the smallest if all are positive, the largest if
 * all are negative, zero otherwise */
double or_minmod3(double a, double b, double c)
{
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}

/* generalized minmod over the backward, central and forward differences */
double or_limited_slope(double dminus, double dplus, double theta)
{
    return or_minmod3(theta * dminus, 0.5 * (dminus + dplus), theta * dplus);
}

/* eq. numerical_flux in the x-direction for the state (eta, p, q) where p is
 * the momentum normal to the face and q the transverse one.  The face depth
 * Hf is shared by both sides, so h^R - h^L = eta^R - eta^L.  Velocities are
 * desingularised (eq. desing_ours) and the momenta recomputed as h*u so that
 * they vanish continuously at dry faces.  The transverse momentum is carried
 * by the mass flux, upwinded by its sign. */
void or_cu_flux(const double *L, const double *R, double Hf, double g, double kappa, double *out)
{
    double hL = L[0] + Hf, hR = R[0] + Hf;
    double sL = or_desing(hL, kappa), sR = or_desing(hR, kappa);
    double uL = L[1] / sL, vL = L[2] / sL;
    double uR = R[1] / sR, vR = R[2] / sR;
    double pL = hL * uL, pR = hR * uR;
    double cL = sqrt(g * fmax(hL, 0.0)), cR = sqrt(g * fmax(hR, 0.0));
    double ap = fmax(fmax(uL + cL, uR + cR), 0.0);
    double am = fmin(fmin(uL - cL, uR - cR), 0.0);
    double FL0 = pL, FL1 = pL * uL + 0.5 * g * hL * hL;
    double FR0 = pR, FR1 = pR * uR + 0.5 * g * hR * hR;
    if (ap - am > 0.0) {
        double w = 1.0 / (ap - am);
        out[0] = (ap * FL0 - am * FR0) * w + ap * am * w * (R[0] - L[0]);
        out[1] = (ap * FL1 - am * FR1) * w + ap * am * w * (pR - pL);
        out[2] = out[0] * (out[0] >= 0.0 ? vL : vR);
    } else {
        out[0] = 0.5 * (FL0 + FR0);
        out[1] = 0.5 * (FL1 + FR1);
        out[2] = 0.5 * (pL * vL + pR * vR);
    }
}

/* ------------------------------------------------------------------------- */
/* forcing: linear interpolation in time (eq. windstress_interpol)           */
/* ------------------------------------------------------------------------- */

static void time_weights(int n, const double *ts, double tau, int *k, double *s)
{
    if (n <= 1 || tau <= ts[0]) { *k = 0; *s = 0.0; return; }
    if (tau >= ts[n - 1]) { *k = n - 2; *s = 1.0; return; }
    int a = 0;
    while (a < n - 2 && ts[a + 1] <= tau) a++;
    *k = a;
    *s = (tau - ts[a]) / (ts[a + 1] - ts[a]);
}

static void wind_at(const or_params *p, double tau, double *tx, double *ty)
{
    int k; double s;
    if (p->wind_n <= 0 || !p->wind_tau) { *tx = *ty = 0.0; return; }
    time_weights(p->wind_n, p->wind_t, tau, &k, &s);
    if (p->wind_n == 1) { *tx = p->wind_tau[0]; *ty = p->wind_tau[1]; return; }
    *tx = (1.0 - s) * p->wind_tau[2 * k] + s * p->wind_tau[2 * (k + 1)];
    *ty = (1.0 - s) * p->wind_tau[2 * k + 1] + s * p->wind_tau[2 * (k + 1) + 1];
}

/* Wind at 10 m from its own grid (section "Wind"): linear in time between
 * the two snapshots around tau (eq. windstress_interpol), bilinear in space
 * with the samples at the centres of a w10_nx x w10_ny partition of the
 * domain and clamped at its edges (what a texture fetch with linear
 * filtering returns), then (w10_kind 0) the stress of Large and Pond,
 *   tau / rho_w = (rho_a / rho_w) C_D |W| W,
 *   C_D = 1.2e-3 for |W| < 11 m/s, (0.49 + 0.065 |W|) 1e-3 above,
 * returned as the kinematic source of the momentum equations. */
static double w10_sample(const or_params *p, int snap, double gx, double gy, int comp)
{
    const int nxw = p->w10_nx, nyw = p->w10_ny;
    if (gx < 0.0) gx = 0.0;
    if (gx > nxw - 1) gx = nxw - 1;
    if (gy < 0.0) gy = 0.0;
    if (gy > nyw - 1) gy = nyw - 1;
    int i0 = (int)floor(gx), j0 = (int)floor(gy);
    int i1 = i0 + 1 < nxw ? i0 + 1 : nxw - 1, j1 = j0 + 1 < nyw ? j0 + 1 : nyw - 1;
    double fx = gx - i0, fy = gy - j0;
    const double *W = p->w10 + (size_t)snap * nxw * nyw * 2;
#define WS(i, j) W[((size_t)(j) * nxw + (i)) * 2 + comp]
    double south = (1.0 - fx) * WS(i0, j0) + fx * WS(i1, j0);
    double north = (1.0 - fx) * WS(i0, j1) + fx * WS(i1, j1);
#undef WS
    return (1.0 - fy) * south + fy * north;
}

static void w10_stress(const or_params *p, int i, int j, double tau, double *sx, double *sy)
{
    *sx = *sy = 0.0;
    if (p->w10_n <= 0 || !p->w10) return;
    int k; double s;
    time_weights(p->w10_n, p->w10_t, tau, &k, &s);
    int kb = p->w10_n > 1 ? k + 1 : k;
    /* cell centre in wind-grid sample coordinates */
    double gx = (i + 0.5) * p->w10_nx / (double)p->nx - 0.5;
    double gy = (j + 0.5) * p->w10_ny / (double)p->ny - 0.5;
    double W[2];
    for (int c = 0; c < 2; ++c)
        W[c] = (1.0 - s) * w10_sample(p, k, gx, gy, c) + s * w10_sample(p, kb, gx, gy, c);
    if (p->w10_kind == 1) {  /* a stress field: interpolated as it is */
        *sx = W[0] / p->rho_w;
        *sy = W[1] / p->rho_w;
        return;
    }
    double speed = sqrt(W[0] * W[0] + W[1] * W[1]);
    double cd = speed < 11.0 ? 1.2e-3 : (0.49 + 0.065 * speed) * 1e-3;
    double q = p->rho_a / p->rho_w * cd * speed;
    *sx = q * W[0];
    *sy = q * W[1];
}

/* external state at perimeter position idx (W: row, E: ny+row, S: 2ny+col,
 * N: 2ny+nx+col) for field fld (0 eta, 1 hu, 2 hv) at time tau */
static double ext_at(const or_params *p, int idx, int fld, double tau)
{
    int P = 2 * p->ny + 2 * p->nx, k; double s;
    time_weights(p->bnd_n, p->bnd_t, tau, &k, &s);
    const double *a = p->bnd + ((size_t)k * 3 + fld) * P;
    if (p->bnd_n == 1) return a[idx];
    const double *b = p->bnd + ((size_t)(k + 1) * 3 + fld) * P;
    return (1.0 - s) * a[idx] + s * b[idx];
}

/* ------------------------------------------------------------------------- */
/* workspace with ghost cells                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nx, ny, sx, csx;
    double *eta, *hu, *hv, *f, *north;   /* cells with NG ghost layers */
    unsigned char *land;
    double *Hc;                          /* corners with NG ghost layers */
    double *h, *hs, *u, *v, *cx, *cy;    /* cell quantities */
    double *eE, *eW, *uE, *uW, *vE, *vW; /* x-face values (eta, hu, hv) */
    double *eN, *eS, *uN, *uS, *vN, *vS; /* y-face values */
    double *F[3];                        /* flux through the east face of each cell */
    double *G[3];                        /* flux through the north face of each cell */
    double *block;
} ws_t;

#define CI(w, i, j) ((size_t)((j) + NG) * (size_t)(w)->sx + (size_t)((i) + NG))
#define KI(w, i, j) ((size_t)((j) + NG) * (size_t)(w)->csx + (size_t)((i) + NG))

static int ws_init(ws_t *w, int nx, int ny)
{
    memset(w, 0, sizeof(*w));
    w->nx = nx; w->ny = ny;
    w->sx = nx + 2 * NG;
    w->csx = nx + 1 + 2 * NG;
    size_t nc = (size_t)w->sx * (size_t)(ny + 2 * NG);
    size_t nk = (size_t)w->csx * (size_t)(ny + 1 + 2 * NG);
    int nplanes = 5 + 6 + 12 + 6;
    w->block = (double *)malloc(sizeof(double) * (nc * (size_t)nplanes + nk));
    w->land = (unsigned char *)calloc(nc, 1);
    if (!w->block || !w->land) { free(w->block); free(w->land); return -2; }
    double *q = w->block;
    double **planes[] = {&w->eta, &w->hu, &w->hv, &w->f, &w->north,
                         &w->h, &w->hs, &w->u, &w->v, &w->cx, &w->cy,
                         &w->eE, &w->eW, &w->uE, &w->uW, &w->vE, &w->vW,
                         &w->eN, &w->eS, &w->uN, &w->uS, &w->vN, &w->vS,
                         &w->F[0], &w->F[1], &w->F[2], &w->G[0], &w->G[1], &w->G[2]};
    for (int k = 0; k < nplanes; ++k) { *planes[k] = q; q += nc; }
    w->Hc = q;
    /* poison everything; only what the cross-shaped stencil needs is filled */
    for (size_t k = 0; k < nc * (size_t)nplanes + nk; ++k) w->block[k] = NAN;
    return 0;
}

static void ws_free(ws_t *w) { free(w->block); free(w->land); }

static int check_params(const or_params *p)
{
    if (p->nx < 1 || p->ny < 1 || !(p->dx > 0) || !(p->dy > 0) || !(p->g > 0) || !(p->kappa > 0))
        return -1;
    if ((p->bc[0] == OR_BC_PERIODIC) != (p->bc[1] == OR_BC_PERIODIC)) return -1;
    if ((p->bc[2] == OR_BC_PERIODIC) != (p->bc[3] == OR_BC_PERIODIC)) return -1;
    for (int k = 0; k < 4; ++k) {
        if (p->bc[k] < 0 || p->bc[k] > 2) return -1;
        if (p->bc[k] == OR_BC_NESTED && (p->bnd_n < 1 || !p->bnd || !p->bnd_t)) return -1;
    }
    if (p->w10_n > 0 && (p->w10_nx < 1 || p->w10_ny < 1 || !p->w10 || !p->w10_t || !(p->rho_a > 0))) return -1;
    if (!(p->dt_interval >= 0.0)) return -1;
    if (p->w10_kind != 0 && p->w10_kind != 1) return -1;
    return 0;
}

/* Ghost cells for the state at time tau.
 * Wall (eq. tradWallBCx + f(-x) = -f(x) from eq. KxWallBCReq): eta, tangential
 *   momentum, north angle and land are mirrored, normal momentum and f are
 *   mirrored with a sign change; depths are mirrored about the wall.
 * Periodic: copied from the opposite side.
 * Nested: the external state Q^ext(tau) of that boundary row/column; f, north
 *   angle and depths are mirrored from the interior without sign change; a
 *   nested ghost is never land. */
static void fill_cells(const or_params *p, const or_static *s, ws_t *w, const double *eta,
                       const double *hu, const double *hv, double tau)
{
    const int nx = p->nx, ny = p->ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t a = (size_t)j * nx + i, b = CI(w, i, j);
            w->eta[b] = eta[a]; w->hu[b] = hu[a]; w->hv[b] = hv[a];
            w->f[b] = s->f[a]; w->north[b] = s->north ? s->north[a] : 0.0;
            w->land[b] = s->land ? (s->land[a] != 0) : 0;
        }
    /* x-sides */
    for (int j = 0; j < ny; ++j)
        for (int gk = 1; gk <= NG; ++gk)
            for (int side = 0; side < 2; ++side) {
                int i = side == 0 ? -gk : nx - 1 + gk;
                int bc = p->bc[side];
                int src = side == 0 ? (bc == OR_BC_PERIODIC ? nx - gk : gk - 1)
                                    : (bc == OR_BC_PERIODIC ? gk - 1 : nx - gk);
                size_t b = CI(w, i, j), a = CI(w, src, j);
                w->north[b] = w->north[a];
                if (bc == OR_BC_NESTED) {
                    int idx = side == 0 ? j : ny + j;
                    w->eta[b] = ext_at(p, idx, 0, tau);
                    w->hu[b] = ext_at(p, idx, 1, tau);
                    w->hv[b] = ext_at(p, idx, 2, tau);
                    w->f[b] = w->f[a];
                    w->land[b] = 0;
                } else {
                    double sg = bc == OR_BC_WALL ? -1.0 : 1.0;
                    w->eta[b] = w->eta[a];
                    w->hu[b] = sg * w->hu[a];
                    w->hv[b] = w->hv[a];
                    w->f[b] = sg * w->f[a];
                    w->land[b] = w->land[a];
                }
            }
    /* y-sides */
    for (int i = 0; i < nx; ++i)
        for (int gk = 1; gk <= NG; ++gk)
            for (int side = 0; side < 2; ++side) {
                int j = side == 0 ? -gk : ny - 1 + gk;
                int bc = p->bc[2 + side];
                int src = side == 0 ? (bc == OR_BC_PERIODIC ? ny - gk : gk - 1)
                                    : (bc == OR_BC_PERIODIC ? gk - 1 : ny - gk);
                size_t b = CI(w, i, j), a = CI(w, i, src);
                w->north[b] = w->north[a];
                if (bc == OR_BC_NESTED) {
                    int idx = side == 0 ? 2 * ny + i : 2 * ny + nx + i;
                    w->eta[b] = ext_at(p, idx, 0, tau);
                    w->hu[b] = ext_at(p, idx, 1, tau);
                    w->hv[b] = ext_at(p, idx, 2, tau);
                    w->f[b] = w->f[a];
                    w->land[b] = 0;
                } else {
                    double sg = bc == OR_BC_WALL ? -1.0 : 1.0;
                    w->eta[b] = w->eta[a];
                    w->hu[b] = w->hu[a];
                    w->hv[b] = sg * w->hv[a];
                    w->f[b] = sg * w->f[a];
                    w->land[b] = w->land[a];
                }
            }
}

/* corner depths with ghost layers: mirrored about wall and nested sides,
 * wrapped for periodic sides (which must then agree on the seam) */
static void fill_corners(const or_params *p, const or_static *s, ws_t *w)
{
    const int nx = p->nx, ny = p->ny;
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) w->Hc[KI(w, i, j)] = s->Hc[(size_t)j * (nx + 1) + i];
    for (int j = 0; j <= ny; ++j)
        for (int gk = 1; gk <= NG; ++gk) {
            int srcW = p->bc[0] == OR_BC_PERIODIC ? nx - gk : gk;
            int srcE = p->bc[1] == OR_BC_PERIODIC ? gk : nx - gk;
            w->Hc[KI(w, -gk, j)] = w->Hc[KI(w, srcW, j)];
            w->Hc[KI(w, nx + gk, j)] = w->Hc[KI(w, srcE, j)];
        }
    for (int i = 0; i <= nx; ++i)
        for (int gk = 1; gk <= NG; ++gk) {
            int srcS = p->bc[2] == OR_BC_PERIODIC ? ny - gk : gk;
            int srcN = p->bc[3] == OR_BC_PERIODIC ? gk : ny - gk;
            w->Hc[KI(w, i, -gk)] = w->Hc[KI(w, i, srcS)];
            w->Hc[KI(w, i, ny + gk)] = w->Hc[KI(w, i, srcN)];
        }
}

/* depth at the west face of cell (i,j) (= H_{i-1/2,j}), at the south face
 * (= H_{i,j-1/2}) and the cell average (mean of the four corners) */
static double Hwest(const ws_t *w, int i, int j) { return 0.5 * (w->Hc[KI(w, i, j)] + w->Hc[KI(w, i, j + 1)]); }
static double Hsouth(const ws_t *w, int i, int j) { return 0.5 * (w->Hc[KI(w, i, j)] + w->Hc[KI(w, i + 1, j)]); }
static double Hbar(const ws_t *w, int i, int j)
{
    return 0.25 * (w->Hc[KI(w, i, j)] + w->Hc[KI(w, i + 1, j)] + w->Hc[KI(w, i, j + 1)] +
                   w->Hc[KI(w, i + 1, j + 1)]);
}

/* h, h*, u, v and the Coriolis terms c_x = f x.(v^n, -u^e), c_y = f y.(v^n, -u^e)
 * with e = (cos, -sin), n = (sin, cos), x = (cos, sin), y = (-sin, cos) */
static void cell_quantities(const or_params *p, ws_t *w, int i, int j)
{
    size_t b = CI(w, i, j);
    double h = w->eta[b] + Hbar(w, i, j);
    double hs = or_desing(h, p->kappa);
    double u = w->hu[b] / hs, v = w->hv[b] / hs;
    double th = w->north[b], c = cos(th), sn = sin(th);
    double ue = c * u - sn * v;
    double vn = sn * u + c * v;
    w->h[b] = h; w->hs[b] = hs; w->u[b] = u; w->v[b] = v;
    w->cx[b] = w->f[b] * (c * vn - sn * ue);
    w->cy[b] = w->f[b] * (-sn * vn - c * ue);
}

/* x-direction slopes and E/W face values of cell (i,j) (eqs. Kbackwards, hE,
 * KxE_adjust).  Slopes are kept in length units: sigma = dx * (slope). */
static void x_faces(const or_params *p, ws_t *w, int i, int j)
{
    size_t b = CI(w, i, j), bm = CI(w, i - 1, j), bp = CI(w, i + 1, j);
    double kx = p->dx / (2.0 * p->g);
    double dm = w->eta[b] - w->eta[bm] - kx * (w->cx[bm] + w->cx[b]);
    double dp = w->eta[bp] - w->eta[b] - kx * (w->cx[b] + w->cx[bp]);
    double sK = or_limited_slope(dm, dp, p->theta);
    double su = or_limited_slope(w->hu[b] - w->hu[bm], w->hu[bp] - w->hu[b], p->theta);
    double sv = or_limited_slope(w->hv[b] - w->hv[bm], w->hv[bp] - w->hv[b], p->theta);
    if (w->land[bm] || w->land[bp]) sK = su = sv = 0.0; /* first order along the shore */
    double rho = 0.5 * sK + kx * w->cx[b];
    double eE = w->eta[b] + rho, eW = w->eta[b] - rho;
    double HE = Hwest(w, i + 1, j), HW = Hwest(w, i, j);
    if (eE + HE < 0.0) { eE = -HE; eW = 2.0 * w->eta[b] - eE; }
    if (eW + HW < 0.0) { eW = -HW; eE = 2.0 * w->eta[b] - eW; }
    w->eE[b] = eE; w->eW[b] = eW;
    w->uE[b] = w->hu[b] + 0.5 * su; w->uW[b] = w->hu[b] - 0.5 * su;
    w->vE[b] = w->hv[b] + 0.5 * sv; w->vW[b] = w->hv[b] - 0.5 * sv;
}

/* y-direction analogue with L = g(eta + U), U_y = (f/g) u, which gives the
 * backward difference eta_j - eta_{j-1} - dy/(2g) (c_y,j-1 + c_y,j) */
static void y_faces(const or_params *p, ws_t *w, int i, int j)
{
    size_t b = CI(w, i, j), bm = CI(w, i, j - 1), bp = CI(w, i, j + 1);
    double ky = p->dy / (2.0 * p->g);
    double dm = w->eta[b] - w->eta[bm] - ky * (w->cy[bm] + w->cy[b]);
    double dp = w->eta[bp] - w->eta[b] - ky * (w->cy[b] + w->cy[bp]);
    double sL = or_limited_slope(dm, dp, p->theta);
    double su = or_limited_slope(w->hu[b] - w->hu[bm], w->hu[bp] - w->hu[b], p->theta);
    double sv = or_limited_slope(w->hv[b] - w->hv[bm], w->hv[bp] - w->hv[b], p->theta);
    if (w->land[bm] || w->land[bp]) sL = su = sv = 0.0;
    double rho = 0.5 * sL + ky * w->cy[b];
    double eN = w->eta[b] + rho, eS = w->eta[b] - rho;
    double HN = Hsouth(w, i, j + 1), HS = Hsouth(w, i, j);
    if (eN + HN < 0.0) { eN = -HN; eS = 2.0 * w->eta[b] - eN; }
    if (eS + HS < 0.0) { eS = -HS; eN = 2.0 * w->eta[b] - eS; }
    w->eN[b] = eN; w->eS[b] = eS;
    w->uN[b] = w->hu[b] + 0.5 * su; w->uS[b] = w->hu[b] - 0.5 * su;
    w->vN[b] = w->hv[b] + 0.5 * sv; w->vS[b] = w->hv[b] - 0.5 * sv;
}

/* flux between a left/lower state and a right/upper state.  A face touching
 * land gets the reflective-wall state of its wet side (zero mass flux); a
 * face between two land cells carries nothing. */
static void face_flux(const double *L0, const double *R0, int landL, int landR, double Hf,
                      const or_params *p, double *out)
{
    double L[3] = {L0[0], L0[1], L0[2]}, R[3] = {R0[0], R0[1], R0[2]};
    if (landL && landR) { out[0] = out[1] = out[2] = 0.0; return; }
    if (landR) { R[0] = L[0]; R[1] = -L[1]; R[2] = L[2]; }
    if (landL) { L[0] = R[0]; L[1] = -R[1]; L[2] = R[2]; }
    or_cu_flux(L, R, Hf, p->g, p->kappa, out);
}

static void compute_rhs(const or_params *p, const or_static *s, ws_t *w, const double *eta,
                        const double *hu, const double *hv, double tau, double *Me, double *Mu,
                        double *Mv, double *faces)
{
    const int nx = p->nx, ny = p->ny;
    fill_cells(p, s, w, eta, hu, hv, tau);
    fill_corners(p, s, w);

#pragma omp parallel for schedule(static)
    for (int j = -NG; j < ny + NG; ++j)
        for (int i = -NG; i < nx + NG; ++i) {
            int gx = i < 0 || i >= nx, gy = j < 0 || j >= ny;
            if (gx && gy) continue; /* diagonal ghosts are never part of the cross stencil */
            cell_quantities(p, w, i, j);
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = -1; i <= nx; ++i) x_faces(p, w, i, j);
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) y_faces(p, w, i, j);

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = -1; i < nx; ++i) {
            size_t a = CI(w, i, j), b = CI(w, i + 1, j);
            double L[3] = {w->eE[a], w->uE[a], w->vE[a]};
            double R[3] = {w->eW[b], w->uW[b], w->vW[b]};
            double out[3];
            face_flux(L, R, w->land[a], w->land[b], Hwest(w, i + 1, j), p, out);
            w->F[0][a] = out[0]; w->F[1][a] = out[1]; w->F[2][a] = out[2];
        }
#pragma omp parallel for schedule(static)
    for (int j = -1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t a = CI(w, i, j), b = CI(w, i, j + 1);
            /* y-direction: normal momentum hv, transverse hu */
            double L[3] = {w->eN[a], w->vN[a], w->uN[a]};
            double R[3] = {w->eS[b], w->vS[b], w->uS[b]};
            double out[3];
            face_flux(L, R, w->land[a], w->land[b], Hsouth(w, i, j + 1), p, out);
            w->G[0][a] = out[0]; w->G[2][a] = out[1]; w->G[1][a] = out[2];
        }

    double tx, ty;
    wind_at(p, tau, &tx, &ty);
    const double g = p->g;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t o = (size_t)j * nx + i, b = CI(w, i, j);
            size_t bw = CI(w, i - 1, j), bs = CI(w, i, j - 1);
            if (faces) {
                size_t P = (size_t)nx * ny;
                double vals[12] = {w->eE[b], w->eW[b], w->eN[b], w->eS[b], w->uE[b], w->uW[b],
                                   w->uN[b], w->uS[b], w->vE[b], w->vW[b], w->vN[b], w->vS[b]};
                for (int k = 0; k < 12; ++k) faces[k * P + o] = vals[k];
            }
            if (w->land[b]) { Me[o] = Mu[o] = Mv[o] = 0.0; continue; }
            double HE = Hwest(w, i + 1, j), HW = Hwest(w, i, j);
            double HN = Hsouth(w, i, j + 1), HS = Hsouth(w, i, j);
            double hE = w->eE[b] + HE, hW = w->eW[b] + HW;
            double hN = w->eN[b] + HN, hS = w->eS[b] + HS;
            double th = w->north[b], c = cos(th), sn = sin(th);
            double hue = c * w->hu[b] - sn * w->hv[b];
            double hvn = sn * w->hu[b] + c * w->hv[b];
            double Cx = w->f[b] * (c * hvn - sn * hue);
            double Cy = w->f[b] * (-sn * hvn - c * hue);
            Me[o] = -(w->F[0][b] - w->F[0][bw]) / p->dx - (w->G[0][b] - w->G[0][bs]) / p->dy;
            double wsx, wsy;
            w10_stress(p, i, j, tau, &wsx, &wsy);
            Mu[o] = -(w->F[1][b] - w->F[1][bw]) / p->dx - (w->G[1][b] - w->G[1][bs]) / p->dy +
                    g / (2.0 * p->dx) * (hE + hW) * (HE - HW) + Cx + tx / p->rho_w + wsx;
            Mv[o] = -(w->F[2][b] - w->F[2][bw]) / p->dx - (w->G[2][b] - w->G[2][bs]) / p->dy +
                    g / (2.0 * p->dy) * (hN + hS) * (HN - HS) + Cy + ty / p->rho_w + wsy;
        }
}

int or_rhs(const or_params *p, const or_static *s, const double *eta, const double *hu,
           const double *hv, double t, double *M_eta, double *M_hu, double *M_hv, double *faces)
{
    int rc = check_params(p);
    if (rc) return rc;
    ws_t w;
    if (ws_init(&w, p->nx, p->ny)) return -2;
    compute_rhs(p, s, &w, eta, hu, hv, t, M_eta, M_hu, M_hv, faces);
    ws_free(&w);
    return 0;
}

/* bed shear stress coefficient S >= 0 so that the source is -S (hu, hv):
 * linear r/h*, quadratic r|u|/h*^2 (eq. swe), Manning g n^2 |u| / h*^(4/3) */
static double friction_of(const or_params *p, double h, double hu, double hv)
{
    if (p->friction == OR_FRIC_NONE) return 0.0;
    double a = fabs(or_desing(h, p->kappa));
    double speed = sqrt(hu * hu + hv * hv) / a;
    switch (p->friction) {
    case OR_FRIC_LINEAR: return p->friction_coeff / a;
    case OR_FRIC_QUADRATIC: return p->friction_coeff * speed / (a * a);
    case OR_FRIC_MANNING:
        return p->g * p->friction_coeff * p->friction_coeff * speed / pow(a, 4.0 / 3.0);
    default: return 0.0;
    }
}

static double cell_hbar(const or_static *s, int nx, int i, int j)
{
    const double *H = s->Hc;
    size_t r0 = (size_t)j * (nx + 1), r1 = (size_t)(j + 1) * (nx + 1);
    return 0.25 * (H[r0 + i] + H[r0 + i + 1] + H[r1 + i] + H[r1 + i + 1]);
}

int or_friction(const or_params *p, const or_static *s, const double *eta, const double *hu,
                const double *hv, double *S)
{
    int rc = check_params(p);
    if (rc) return rc;
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            size_t o = (size_t)j * p->nx + i;
            S[o] = (s->land && s->land[o]) ? 0.0
                                           : friction_of(p, eta[o] + cell_hbar(s, p->nx, i, j), hu[o], hv[o]);
        }
    return 0;
}

/* eq. cfl: dt = C * 1/4 * min over non-land cells of min(dx/(|u|+c), dy/(|v|+c)) */
double or_cfl_dt(const or_params *p, const or_static *s, const double *eta, const double *hu,
                 const double *hv)
{
    double best = INFINITY;
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            size_t o = (size_t)j * p->nx + i;
            if (s->land && s->land[o]) continue;
            double h = eta[o] + cell_hbar(s, p->nx, i, j);
            double hs = or_desing(h, p->kappa);
            double c = sqrt(p->g * fmax(h, 0.0));
            double ax = fabs(hu[o] / hs) + c, ay = fabs(hv[o] / hs) + c;
            if (ax > 0.0) best = fmin(best, p->dx / ax);
            if (ay > 0.0) best = fmin(best, p->dy / ay);
        }
    return p->courant * 0.25 * best;
}

/* eq. frs: inside the relaxation zone of width W next to a nested side,
 * Q = (1 - alpha) Q + alpha Q^ext with alpha = 1 - tanh(d/d0), d the distance
 * in cells to that side (0 for the outermost interior cell).  The nearest
 * nested side is used; ties go to W, E, S, N in that order. */
static void apply_frs(const or_params *p, const or_static *s, double *eta, double *hu, double *hv,
                      double tau)
{
    const int nx = p->nx, ny = p->ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t o = (size_t)j * nx + i;
            if (s->land && s->land[o]) continue;
            int dist[4] = {i, nx - 1 - i, j, ny - 1 - j};
            int idxs[4] = {j, ny + j, 2 * ny + i, 2 * ny + nx + i};
            int best = -1, d = 0;
            for (int k = 0; k < 4; ++k)
                if (p->bc[k] == OR_BC_NESTED && (best < 0 || dist[k] < d)) { best = k; d = dist[k]; }
            if (best < 0 || d >= p->frs_width) continue;
            double alpha = 1.0 - tanh((double)d / p->frs_d0);
            int idx = idxs[best];
            eta[o] = (1.0 - alpha) * eta[o] + alpha * ext_at(p, idx, 0, tau);
            hu[o] = (1.0 - alpha) * hu[o] + alpha * ext_at(p, idx, 1, tau);
            hv[o] = (1.0 - alpha) * hv[o] + alpha * ext_at(p, idx, 2, tau);
        }
}

static int any_nested(const or_params *p)
{
    for (int k = 0; k < 4; ++k)
        if (p->bc[k] == OR_BC_NESTED) return 1;
    return 0;
}

typedef struct {
    ws_t w;
    double *M[3], *S, *q1[3], *buf;
} step_ws;

static int step_ws_init(step_ws *sw, int nx, int ny)
{
    if (ws_init(&sw->w, nx, ny)) return -2;
    size_t n = (size_t)nx * ny;
    sw->buf = (double *)malloc(sizeof(double) * n * 7);
    if (!sw->buf) { ws_free(&sw->w); return -2; }
    for (int k = 0; k < 3; ++k) { sw->M[k] = sw->buf + k * n; sw->q1[k] = sw->buf + (3 + k) * n; }
    sw->S = sw->buf + 6 * n;
    return 0;
}

static void step_ws_free(step_ws *sw) { ws_free(&sw->w); free(sw->buf); }

/* eq. rk2_semiimp:
 *   Q*      = (Q^n + dt M(Q^n)) / (1 + dt S(Q^n))             (momenta only)
 *   Q^{n+1} = 1/2 (Q^n + Q* + dt M(Q*)) / (1 + dt/2 S(Q*))     (momenta only)
 * stage 1 evaluated at t^n, stage 2 at t^n + dt, then the FRS nesting at
 * t^{n+1}.  Land cells are frozen. */
static void do_step(const or_params *p, const or_static *s, step_ws *sw, double *eta, double *hu,
                    double *hv, double t, double dt)
{
    const size_t n = (size_t)p->nx * p->ny;
    double *e1 = sw->q1[0], *u1 = sw->q1[1], *v1 = sw->q1[2];
    or_friction(p, s, eta, hu, hv, sw->S);
    compute_rhs(p, s, &sw->w, eta, hu, hv, t, sw->M[0], sw->M[1], sw->M[2], NULL);
    for (size_t o = 0; o < n; ++o) {
        if (s->land && s->land[o]) { e1[o] = eta[o]; u1[o] = hu[o]; v1[o] = hv[o]; continue; }
        double den = 1.0 + dt * sw->S[o];
        e1[o] = eta[o] + dt * sw->M[0][o];
        u1[o] = (hu[o] + dt * sw->M[1][o]) / den;
        v1[o] = (hv[o] + dt * sw->M[2][o]) / den;
    }
    or_friction(p, s, e1, u1, v1, sw->S);
    compute_rhs(p, s, &sw->w, e1, u1, v1, t + dt, sw->M[0], sw->M[1], sw->M[2], NULL);
    for (size_t o = 0; o < n; ++o) {
        if (s->land && s->land[o]) continue;
        double den = 1.0 + 0.5 * dt * sw->S[o];
        eta[o] = 0.5 * (eta[o] + (e1[o] + dt * sw->M[0][o]));
        hu[o] = 0.5 * (hu[o] + (u1[o] + dt * sw->M[1][o])) / den;
        hv[o] = 0.5 * (hv[o] + (v1[o] + dt * sw->M[2][o])) / den;
    }
    if (any_nested(p)) apply_frs(p, s, eta, hu, hv, t + dt);
}

int or_step(const or_params *p, const or_static *s, double *eta, double *hu, double *hv,
            double *t, double dt)
{
    int rc = check_params(p);
    if (rc) return rc;
    step_ws sw;
    if (step_ws_init(&sw, p->nx, p->ny)) return -2;
    do_step(p, s, &sw, eta, hu, hv, *t, dt);
    *t += dt;
    step_ws_free(&sw);
    return 0;
}

int64_t or_run(const or_params *p, const or_static *s, double *eta, double *hu, double *hv,
               double *t, int64_t nsteps, double t_end, double dt_fixed, const double *dts,
               double *dts_out)
{
    int rc = check_params(p);
    if (rc) return rc;
    step_ws sw;
    if (step_ws_init(&sw, p->nx, p->ny)) return -2;
    int64_t k = 0;
    double dt_hold = 0.0, t_upd = *t;  /* dt update policy state */
    for (; k < nsteps; ++k) {
        double dt;
        if (dt_fixed > 0.0) dt = dt_fixed;
        else if (dts) dt = dts[k];
        else {
            if (p->dt_interval > 0.0 && dt_hold > 0.0 && *t < t_upd) {
                dt = dt_hold;
            } else {
                dt = or_cfl_dt(p, s, eta, hu, hv);
                if (p->dt_interval > 0.0) {
                    dt_hold = dt;
                    t_upd += p->dt_interval;
                    if (t_upd <= *t) t_upd = *t + p->dt_interval;
                }
            }
            if (t_end > 0.0) {
                if (*t >= t_end) break;
                if (dt > t_end - *t) dt = t_end - *t;
            }
        }
        if (!isfinite(dt) || !(dt > 0.0)) { step_ws_free(&sw); return -3; }
        do_step(p, s, &sw, eta, hu, hv, *t, dt);
        if (t_end > 0.0 && dt_fixed <= 0.0 && !dts && *t + dt >= t_end) *t = t_end;
        else *t += dt;
        if (dts_out) dts_out[k] = dt;
    }
    step_ws_free(&sw);
    return k;
}

void or_diagnostics(const or_params *p, const or_static *s, const double *eta, const double *hu,
                    const double *hv, double *mass, double *energy)
{
    double m = 0.0, e = 0.0, area = p->dx * p->dy;
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            size_t o = (size_t)j * p->nx + i;
            if (s->land && s->land[o]) continue;
            double h = eta[o] + cell_hbar(s, p->nx, i, j);
            double hs = or_desing(h, p->kappa);
            m += h * area;
            e += (0.5 * (hu[o] * hu[o] + hv[o] * hv[o]) / hs + 0.5 * p->g * eta[o] * eta[o]) * area;
        }
    *mass = m;
    *energy = e;
}
