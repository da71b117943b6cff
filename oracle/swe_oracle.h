/*
 * Plain FP64 CPU oracle for one SSP-RK2 step of the eta-based, well-balanced
 * central-upwind (CDKLM) scheme for the rotational shallow-water equations,
 * as extended in Brodtkorb & Holm, "Real-World Oceanographic Simulations on
 * the GPU using a Two-Dimensional Finite-Volume Scheme" (arXiv 1912.02457).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP implementation.
 *
 * Arrays: cell fields [ny][nx] (x fastest), corner depths [ny+1][nx+1],
 * boundary snapshots [n][3][2ny+2nx] (W strip by row, E strip, S strip by
 * column, N strip), wind snapshots [n][2] in N/m^2, optional gridded wind at
 * 10 m [n][ny_w][nx_w][2] in m/s.  All in float64.
 */
#ifndef SWE_ORACLE_H
#define SWE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BC_WALL = 0, OR_BC_PERIODIC = 1, OR_BC_NESTED = 2 };
enum { OR_FRIC_NONE = 0, OR_FRIC_LINEAR = 1, OR_FRIC_QUADRATIC = 2, OR_FRIC_MANNING = 3 };

typedef struct {
    int32_t nx, ny;
    double dx, dy, g;
    double courant;     /* dt = courant * 1/4 * min(dx/(|u|+c), dy/(|v|+c)) */
    double theta;       /* generalized-minmod parameter */
    double kappa;       /* desingularisation / dry tolerance (m) */
    int32_t bc[4];      /* W, E, S, N */
    int32_t friction;   /* OR_FRIC_* */
    double friction_coeff;
    double rho_w;
    int32_t frs_width;
    double frs_d0;
    int32_t wind_n;     /* >= 1 */
    const double *wind_t, *wind_tau;
    int32_t bnd_n;      /* 0 if no nested side */
    const double *bnd_t, *bnd;
    /* wind at 10 m on its own grid (section "Wind"): w10_n snapshots of
     * w10_ny x w10_nx samples of (u, v) in m/s, [n][ny][nx][2]; 0 = none */
    int32_t w10_n, w10_nx, w10_ny;
    const double *w10_t, *w10;
    double rho_a;       /* density of air */
    /* time-step update policy of section "Real-world simulations": 0 = the
     * CFL dt every step; > 0 = the CFL dt only at the first step starting at
     * or after each update time (the run's start, then one interval later
     * each time), the last update's dt in between */
    double dt_interval;
    /* what the gridded field holds: 0 = wind at 10 m in m/s, the stress of
     * Large and Pond taken from the wind interpolated to each cell; 1 = wind
     * stress in N/m^2 at the samples, interpolated as it is */
    int32_t w10_kind;
} or_params;

/* per-cell inputs of the problem statement */
typedef struct {
    const double *Hc;         /* [ny+1][nx+1] */
    const uint8_t *land;      /* [ny][nx] or NULL */
    const double *f;          /* [ny][nx] */
    const double *north;      /* [ny][nx] angle theta, north = (sin, cos) */
} or_static;

/* elementary definitions */
double or_desing(double h, double kappa);
double or_minmod3(double a, double b, double c);
double or_limited_slope(double dminus, double dplus, double theta);
/* x-direction central-upwind flux; L, R = (eta, normal momentum, transverse
 * momentum) at the face, Hf = face depth; out = (F_eta, F_normal, F_trans) */
void or_cu_flux(const double *L, const double *R, double Hf, double g, double kappa, double *out);

/* right-hand side M(Q, t) without bed friction, plus (optionally) the face
 * values: faces = 12 planes [etaE, etaW, etaN, etaS, huE, huW, huN, huS,
 * hvE, hvW, hvN, hvS] each [ny][nx].  Returns 0 or a negative code. */
int or_rhs(const or_params *p, const or_static *s, const double *eta, const double *hu,
           const double *hv, double t, double *M_eta, double *M_hu, double *M_hv, double *faces);

/* friction coefficient S(Q) >= 0 per cell */
int or_friction(const or_params *p, const or_static *s, const double *eta, const double *hu,
                const double *hv, double *S);

/* CFL time step from the state (courant included).  Returns +inf if no
 * non-land cell carries a wave. */
double or_cfl_dt(const or_params *p, const or_static *s, const double *eta, const double *hu,
                 const double *hv);

/* one SSP-RK2 step with semi-implicit friction and FRS nesting, dt given.
 * State is updated in place, *t advanced. */
int or_step(const or_params *p, const or_static *s, double *eta, double *hu, double *hv,
            double *t, double dt);

/* nsteps steps.  dt_fixed > 0: that dt every step; dts != NULL and
 * dt_fixed <= 0: replay dts[k]; otherwise dt from the CFL condition of the
 * state at the start of each step (or at update steps only, under the
 * dt_interval policy), clamped so that t never exceeds t_end
 * when t_end > 0 (the run stops once t reaches t_end).  dts_out (optional)
 * receives the dt of each step.  Returns the number of steps taken, or a
 * negative code. */
int64_t or_run(const or_params *p, const or_static *s, double *eta, double *hu, double *hv,
               double *t, int64_t nsteps, double t_end, double dt_fixed, const double *dts,
               double *dts_out);

/* FP64 mass sum (eta + Hbar) dx dy and energy sum (|hu|^2/(2 h*) + g eta^2/2) dx dy
 * over non-land cells */
void or_diagnostics(const or_params *p, const or_static *s, const double *eta, const double *hu,
                    const double *hv, double *mass, double *energy);

int or_num_threads(void);
void or_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
