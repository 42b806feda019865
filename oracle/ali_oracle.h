/*
 * ali_oracle.h -- plain, slow, FP64 CPU oracle for the ALI-FMM travel-time method
 * (Ludlam, Tant, Dolean, Curtis, "Travel times and ray paths for acoustic and elastic
 * waves in generally anisotropic media", arXiv 2302.10988).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  The GPU product path shares no code with
 * it and must never call it.
 *
 * Conventions (used by every function below):
 *   - grid nodes (i, j): i = x column 0..nx-1, j = z row 0..nz-1 (z = depth); spacing h [m];
 *     linear index idx = j*nx + i; arrays are row-major [nz][nx].
 *   - orientation theta [rad] = angle of the transversely-isotropic symmetry axis measured
 *     from +x toward +z.  The paper's velocity-curve angle is measured from the c22 axis
 *     (perpendicular to the symmetry axis), i.e. the paper's theta_D = theta + 90 deg.
 *   - material record: stiffness [Pa] in the axis frame ("1" = in-plane direction
 *     perpendicular to the axis, "3" = the axis) and density [kg/m^3].  In the paper's
 *     YZ-plane notation (Section 3.2): c22 <- c11, c23 <- c13, c33 <- c33, c44 <- c55.
 *   - travel times in seconds, +INFINITY where a node is unreached.
 *
 * Functions marked "parity unpinned" in the comments implement readings of the paper that
 * no printed value fixes; they are pinned only by invariants (see the test suite).
 */
#ifndef ALI_ORACLE_H
#define ALI_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* wave: OR_WAVE_QP (in-plane quasi-P, the paper's mode) or OR_WAVE_SH (the shear wave
   polarised normal to the plane, Section 6's extension); one value for every material of
   a solve. */
enum { OR_WAVE_QP = 0, OR_WAVE_SH = 1 };
/* vtab: 0 = speeds from the Christoffel equation at run time; 1 = the paper's velocity
   table: the phase speed from the exact speeds at whole degrees of the phase angle and the
   group speed from those at whole degrees of the group angle, linearly interpolated
   (Section 3.2 and Table 3's two ALI-FMM rows). */
typedef struct {
    double c11, c13, c33, c55, c44, c66, rho;
    int32_t wave;
    int32_t vtab;
    int32_t grule;      /* group speed of the straight rays: OR_GROUP_EXACT, or OR_GROUP_PAPER
                           for the paper's run-time inversion (Section 3.2), a second reading
                           used only to test which rule the printed errors of Table 3 follow */
    int32_t pad;
} or_material;

enum { OR_GROUP_EXACT = 0, OR_GROUP_PAPER = 1 };

/* Alternative readings of the update and the choice, switched on per thread only by the
   test that measures which readings reproduce the printed errors of Table 3:
     MIN_UPDATE           a close node keeps the smaller of its old and new estimates (the
                          usual Fast Marching rule) instead of being recomputed;
     UNIT_SQUARES_FIRST   the side-1 squares rank before the side-sqrt(2) squares;
     TRIANGLE_LITERAL     the first member of a triangular pair is scored with its own B and
                          C in the second member's formula;
     NO_CAUSALITY         a stencil estimate need not exceed tau_C. */
enum { OR_VAR_MIN_UPDATE = 1, OR_VAR_UNIT_SQUARES_FIRST = 2, OR_VAR_TRIANGLE_LITERAL = 4,
       OR_VAR_NO_CAUSALITY = 8 };
void or_set_reading_variant(int v);

/* ---- Section 3: velocities ------------------------------------------------------- */

/* qP phase speed [m/s] at phase angle th_p [rad] measured from the c22 axis
   (largest root of the in-plane Christoffel matrix, Section 3.2). */
double or_qp_phase_speed(const or_material* m, double th_p);

/* qP group velocity for phase angle th_p (Section 3.1, group velocity from the
   polarisation vector and the stiffness tensor).  Outputs the group angle [rad] from the
   c22 axis and the group speed [m/s]. */
void or_qp_group_from_phase(const or_material* m, double th_p, double* g_angle, double* g_speed);

/* derivative of the qP phase speed with respect to th_p (closed form). */
double or_qp_phase_speed_deriv(const or_material* m, double th_p);

/* derivative of the qP group speed with respect to the group angle (numerical). */
double or_qp_group_speed_deriv(const or_material* m, double phi);

/* qP group speed [m/s] along group angle phi [rad] from the c22 axis, by inverting the
   phase->group angle map with bisection (exact to rounding). */
double or_qp_group_speed(const or_material* m, double phi);

/* The qP group speed as Section 3.2 computes it at run time: the phase angle is the one
   whose qP polarisation points along the group angle phi (the eigenvector condition
   (M - lambda I) X = 0 with X along phi, solved through tan of the phase angle), the
   eigenvalue lambda gives the phase speed v, and the group speed is v / cos(theta - phi).
   Polarisation and group directions differ in a generally anisotropic medium, so this is
   an approximation (up to 0.43 % faster than the exact group speed for the paper's cubic
   steel); it is never used unless a material asks for it (grule). */
double or_qp_group_speed_paper(const or_material* m, double phi);

/* Same quantity by a second, independent route: the support function of the slowness
   curve, 1/V(phi) = max_psi cos(phi - psi) / v(psi). */
double or_qp_group_speed_support(const or_material* m, double phi);

/* SH phase speed at phase angle th_p from the c22 axis: rho v^2 = c66 cos^2 + c44 sin^2
   (the out-of-plane entry of the Christoffel matrix), and its derivative. */
double or_sh_phase_speed(const or_material* m, double th_p);
double or_sh_phase_speed_deriv(const or_material* m, double th_p);

/* SH group speed along group angle phi from the c22 axis: the wave surface of an
   elliptical slowness curve is the ellipse with semi-axes sqrt(c66/rho) (c22 axis) and
   sqrt(c44/rho) (symmetry axis); and its derivative in phi. */
double or_sh_group_speed(const or_material* m, double phi);
double or_sh_group_speed_deriv(const or_material* m, double phi);

/* The speeds of the material's wave (qP or SH by m->wave); every solver below uses these. */
double or_phase_speed(const or_material* m, double th_p);
double or_phase_speed_deriv(const or_material* m, double th_p);
double or_group_speed(const or_material* m, double phi);
double or_group_speed_deriv(const or_material* m, double phi);
/* support-function route for the material's wave (see or_qp_group_speed_support) */
double or_group_speed_support(const or_material* m, double phi);

/* ---- Section 4.1: stencil table --------------------------------------------------- */

/* Offsets (di, dj) of A, B, C relative to D for stencil s = 0..31 (0 = "1-1", 1 = "1-2",
   ..., 31 = "16-2"), with the two printing errors of Table 1 corrected. */
void or_stencil_offsets(int s, int out[6]);

/* ---- Section 4.2: one stencil's estimate ----------------------------------------- */

/* Travel-time estimate at D from the stencil whose support has offsets (xa,ya),(xb,yb),
   (xc,yc) relative to D (grid units), travel times ta < tb <= tc, material m, axis angle
   theta_ax at D, spacing h.  Returns tau_B + |FD| / v(theta'). */
double or_stencil_estimate(const or_material* m, double theta_ax, double h,
                           const int off[6], double ta, double tb, double tc);

/* ---- Section 4.3: stencil choice Phi_D(K) ----------------------------------------- */

/* Estimate at node (i, j) from the set K of known diamond neighbours given by
   known[] (nonzero = known; array over the whole grid).  Returns the value and, through
   choice (nullable), the chosen candidate: 0..31 = stencil, 32 + k = straight-ray
   fallback from the k-th 8-neighbour, -1 = none (value +inf).  parity unpinned (reading). */
double or_phi_d(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                const double* orient, const double* T, const uint8_t* known,
                int i, int j, int* choice);

/* ---- Section 2 / 4.4: drivers ------------------------------------------------------ */

/* Straight-ray source box (Section 4.4 first paragraph): for every node within Chebyshev
   radius R of the source node (si, sj), T = |N - S| h / V_group(direction) with the
   source node's material and orientation.  Writes T and sets fixed[] for those nodes. */
void or_source_box(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                   const double* orient, int si, int sj, int R, double* T, uint8_t* fixed);

/* Heap-based Fast Marching (Section 2) with the ALI update.  T[nz*nx] out.
   pop_order (nullable, length nx*nz) receives the linear index of each popped node in
   pop order; returns the number of pops (or -1 on invalid input). */
int64_t or_solve_fmm(int nx, int nz, double h, const or_material* mats, int n_mats,
                     const uint8_t* mat_id, const double* orient, int si, int sj, int R,
                     double* T, int64_t* pop_order, double* pop_values);

/* Heap Fast Marching from a seeded set: fixed[] marks the nodes whose T is given (all
   other T are overwritten).  With stop_r >= 0 the march ends at the first accepted node
   farther than stop_r (Chebyshev) from (ci, cj); its time goes to *t_stop (+inf if the
   march ran to the end).  known[] receives the accepted nodes.  Returns the number of
   accepted nodes, or -1 on invalid input. */
int64_t or_fmm_seeded(int nx, int nz, double h, const or_material* mats, int n_mats, const uint8_t* mat_id,
                      const double* orient, const uint8_t* fixed, double* T, int ci, int cj, int stop_r,
                      uint8_t* known, double* t_stop);

/* Nested fine grids around the source (Section 4.4): n_levels grids of density[l] nodes
   per spacing (odd, each divisible by the next) used out to radius[l] cells (Chebyshev,
   increasing), then the grid itself; straight rays in the square of half-width vor_half
   cells around the source on the finest grid.  T[nz*nx] out.  Returns 0 or -1.
   parity unpinned beyond the accuracy pins (readings). */
int or_solve_refined(int nx, int nz, double h, const or_material* mats, int n_mats, const uint8_t* mat_id,
                     const double* orient, int si, int sj, int n_levels, const int* density,
                     const int* radius, double vor_half, double* T);

/* Number of Phi_D evaluations made by the last or_solve_fmm call (statistics). */
int64_t or_last_phi_evals(void);

/* The local operator whose unique fixed point is the heap result: value at non-fixed
   node (i, j) computed from the current field T only (neighbours sorted by (T, idx), the
   known set grown in that order, stop once the estimate is below the next neighbour). */
double or_localfmm(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                   const double* orient, const double* T, int i, int j, int* choice);

/* Independent driver: Gauss-Seidel sweeps of or_localfmm to a bitwise fixed point.
   Returns the number of sweeps, or -1 if max_sweeps was reached. */
int or_sweep_solve(int nx, int nz, double h, const or_material* mats, int n_mats,
                   const uint8_t* mat_id, const double* orient, int si, int sj, int R,
                   int max_sweeps, double* T);

/* Dense-stencil Dijkstra reference: edges to every node within Euclidean radius rad
   (grid units); edge time = exact cell-walk of the straight segment through the
   nearest-node cells at group speed.  Source at node (si, sj) with T = 0. */
void or_dijkstra_dense(int nx, int nz, double h, const or_material* mats,
                       const uint8_t* mat_id, const double* orient, int si, int sj,
                       double rad, double* T);

/* Straight-segment travel time from point p0 to p1 (grid coordinates) through the
   nearest-node cells at group speed (the segment time used by the ray tracer). */
double or_segment_time(int nx, int nz, double h, const or_material* mats,
                       const uint8_t* mat_id, const double* orient,
                       double x0, double z0, double x1, double z1);

/* ---- Section 5.1: ray tracing ------------------------------------------------------ */

/* Ray from node (ri, rj) to the source (si, sj) of field T (reciprocity).  Candidates
   are spaced 1/sub node spacing within +-window nodes of the straight-ahead point.  Writes
   up to max_pts points (x, z in grid units) to pts[2*max_pts], their number to *n_pts
   and the integrated time to *t_ray.  Returns 0 on success, -1 if S was not reached. */
int or_trace_ray(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                 const double* orient, const double* T, int si, int sj, int ri, int rj,
                 int window, int sub, int max_pts, double* pts, int* n_pts, double* t_ray);

/* Same with the plane family fixed for the whole ray (family 0: x = k, 1: z = k,
   2: x + z = k, 3: x - z = k; -1: the changing family of or_trace_ray). */
int or_trace_ray_family(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                        const double* orient, const double* T, int si, int sj, int ri, int rj, int family,
                        int window, int sub, int max_pts, double* pts, int* n_pts, double* t_ray);

/* ---- gradient with respect to orientation (frozen choices) --------------------------- */

/* partial derivatives of or_stencil_estimate with respect to ta, tb, tc and theta_ax, and
   (dA nullable, 4 values) with respect to A11, A13, A33, A55 of the node's material, where
   A = C / rho is the density-normalised stiffness */
void or_stencil_partials(const or_material* m, double theta_ax, double h, const int off[6],
                         double ta, double tb, double tc, double* dta, double* dtb, double* dtc,
                         double* dth, double* dA);

/* d v / d (A11, A13, A33, A55) of the qP phase speed at phase angle th_p (closed form,
   eigenvalue perturbation of the Christoffel matrix) */
void or_qp_phase_speed_dA(const or_material* m, double th_p, double dv[4]);

/* d V / d (A11, A13, A33, A55) of the qP group speed at fixed group angle phi (numerical) */
void or_qp_group_speed_dA(const or_material* m, double phi, double dV[4]);

/* choice of every node at the fixed point T: -2 fixed, -1 unreached, 0..31 stencil,
   32 + k straight ray from the k-th 8-neighbour */
void or_field_choices(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                      const double* orient, const double* T, const uint8_t* fixed, int* choice);

/* field recomputed in pop order with frozen choices (orientation may be perturbed) */
void or_frozen_field(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                     const double* orient, int si, int sj, int R, const int* choice,
                     const int64_t* pop, int64_t npop, double* T);

/* dL/dtheta for one source given g = dL/dT at every node; writes the field to T_out
   (nullable) and dL/dA [nz][nx][4] (A11, A13, A33, A55 of every node, A = C / rho; nullable;
   qP only) to dA.  Returns 0, or -1 on invalid input. */
int or_adjoint(int nx, int nz, double h, const or_material* mats, int n_mats, const uint8_t* mat_id,
               const double* orient, int si, int sj, int R, const double* g, double* T_out,
               double* dtheta, double* dA);

#ifdef __cplusplus
}
#endif
#endif
