/*
 * rtgd_oracle.h -- plain FP64 CPU oracle for batched HF ray tracing through a
 * Galerkin-Difference (GD, p = 3) interpolated electron-density grid.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library; its structs
 * are its own.
 *
 * Method (paper: "Efficient and High-Accuracy Ray Tracing in Discretized
 * Ionospheric Models", RTM-GD):
 *   - ray equations: Sec. II-A, eq. (1a)-(1f), with the frame term of (1d)
 *     read as k_phi*sin(theta)*dphi/dP' (the printed form omits sin(theta);
 *     without it dH/dP' != 0);
 *   - Hamiltonian: Sec. II-A, eq. (hamiltonian), Appleton-Hartree
 *     refractive index eq. (appleton), collisionless, + = O, - = X;
 *   - GD interpolant: Sec. II-B-2, eq. (3dinterp_gd) with the p = 3 pieces
 *     of Appendix A (four quintics per cell, 4x4x4 nodes);
 *   - algorithm: Sec. II-C (initialise, per step GD -> refractive index ->
 *     Hamiltonian -> RK4, until ground return or exit).
 *
 * Units: lengths in km, angles in degrees at the interface and radians
 * inside, frequency in MHz, electron density in m^-3, field in tesla.
 * The wave-normal vector is n = c k / omega (dimensionless, |n| = mu).
 * Coordinates: r (geocentric radius), theta (colatitude), phi (east
 * longitude); theta-hat points south.
 */
#ifndef RTGD_ORACLE_H
#define RTGD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* medium kinds */
#define OR_GRID 0      /* GD p=3 interpolation of a gridded N_e               */
#define OR_CHAPMAN 1   /* analytic alpha-Chapman layer (pins only)             */
#define OR_QP 2        /* analytic quasi-parabolic layer (pins only)           */
#define OR_GRID_CR 3   /* Catmull-Rom tensor interpolation of the same grid    */

/* per-ray termination status */
#define OR_GROUND 0
#define OR_ESCAPE 1
#define OR_MAX_PATH 2
#define OR_NUMERIC 3

typedef struct {
    int kind;
    int n_lat, n_lon, n_h;
    double lat0_deg, dlat_deg;   /* first latitude node, spacing            */
    double lon0_deg, dlon_deg;   /* first longitude node, spacing           */
    double h0_km, dh_km;         /* first height node (grid bottom), spacing */
    const double *ne;            /* N_e in m^-3, C order [n_lat][n_lon][n_h] */
    double fc_mhz;               /* analytic layers: critical frequency      */
    double hm_km;                /* analytic layers: peak height             */
    double thick_km;             /* Chapman scale height H / QP semi-thickness */
    double floor_km;             /* N_e = 0 below this height (vacuum)       */
} or_medium;

typedef struct {
    double B0_T;                 /* axial centred dipole strength; 0 = none  */
} or_field;

typedef struct {
    double R_km;                 /* spherical Earth radius                   */
    double tx_lat_deg, tx_lon_deg, tx_h_km;
    double step_km;              /* fixed RK4 step in group path             */
    double max_group_km;         /* MAX_PATH limit                           */
    double exit_h_km;            /* ESCAPE height                            */
    int traj_stride;             /* 0 = no trajectory                        */
    int nthreads;                /* 0 = OpenMP default                       */
} or_opts;

/* Hamiltonian and its partial derivatives at one state. */
typedef struct {
    double H;        /* 0.5 (n.n - mu^2)                                    */
    double G;        /* omega dH/domega at fixed k                          */
    double Hn[3];    /* dH/dn_r, dH/dn_theta, dH/dn_phi                     */
    double Hq[3];    /* dH/dr, dH/dtheta, dH/dphi at fixed local n          */
    double X;        /* f_N^2 / f^2                                         */
    double mu2;      /* Appleton-Hartree mu^2                               */
} or_ham;

/* 1-D GD p=3 weights w_a(s) and dw_a/ds for node offsets a = -1, 0, 1, 2. */
void or_gd_weights(double s, double w[4], double dw[4]);

/* 1-D Catmull-Rom weights, same node offsets. */
void or_cr_weights(double s, double w[4], double dw[4]);

/* N_e and its partials dNe/dr, dNe/dtheta, dNe/dphi at (r, theta, phi). */
void or_medium_eval(const or_medium *m, double R_km, double r, double th,
                    double ph, double out[4]);

/* Dipole gyro-frequency ratio vector Y (local r, theta, phi components)
 * and its r- and theta-derivatives, for frequency f. */
void or_dipole(double B0_T, double R_km, double f_mhz, double r, double th,
               double Y[3], double dYdr[3], double dYdth[3]);

/* Appleton-Hartree mu^2 and its partials with respect to (X, a = Y_T^2,
 * b = Y_L^2) treated as independent; mode > 0 = O, mode < 0 = X. */
int or_appleton(double X, double a, double b, int mode, double out[4]);

/* Hamiltonian, G and partials at state y = (r, th, ph, n_r, n_th, n_ph). */
int or_hamiltonian(const or_medium *m, const or_field *fld, double R_km,
                   double f_mhz, int mode, const double y[6], or_ham *out);

/* Right-hand side dy/dP' of the 7-component state (6 + phase path). */
int or_rhs(const or_medium *m, const or_field *fld, double R_km,
           double f_mhz, int mode, const double y[7], double dy[7]);

/* Launch: vacuum straight line from the transmitter to the medium floor.
 * Writes the 7-component state and returns the vacuum path length. */
double or_launch(const or_opts *o, double floor_km, double elev_deg,
                 double az_deg, double y[7]);

/* Trace n rays.  out7[i*7 + k], k = group, phase, ground range (km),
 * azimuth deviation (deg), apogee (km), landing lat, landing lon (deg).
 * traj (may be NULL): per ray traj_per_ray records of 8 doubles
 * (r, th, ph, n_r, n_th, n_ph, P', P) at steps 0, stride, 2 stride, ...
 * and at the last step; traj_count[i] records written (capped).
 * Returns the total number of RK4 steps taken. */
long long or_trace(const or_medium *m, const or_field *fld, const or_opts *o,
                   int n, const double *elev_deg, const double *az_deg,
                   const double *f_mhz, const int *mode, double *out7,
                   int *status, int *n_steps, double *traj, int traj_per_ray,
                   int *traj_count);

#ifdef __cplusplus
}
#endif
#endif
