/*
 * Plain FP64 CPU oracle for one explicit SSP-RK(2,2) step of the cell-centred
 * finite-volume scheme for the 2D nonlinear shallow water equations
 * (Sections 2.1-2.5 of Giles et al., "Performance analysis of Volna-OP2").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code with the GPU library: it builds its own edge table, neighbours,
 * geometry and orientation from the raw (vertices, triangles, depth) input.
 *
 * No blocking, no fusion: a cell loop for the reconstruction, an edge loop
 * for the fluxes (stored per edge side), a cell loop that accumulates each
 * cell's three faces in local order and applies the Runge-Kutta stage.  The
 * loops may run on several OpenMP threads (orc_set_threads); every
 * iteration writes only its own outputs and the reductions (CFL minimum,
 * clamp count) are exact, so results are bitwise independent of the thread
 * count.
 */
#ifndef VSW_ORACLE_H
#define VSW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_mesh orc_mesh;

typedef struct orc_params {
    double g;            /* gravity, m/s^2 */
    double cfl;          /* Courant number of the dt rule */
    double h_threshold;  /* H_thr, m (Section 2.4) */
    double dt_fixed;     /* > 0: constant dt; 0: CFL rule */
} orc_params;

/* Build connectivity and geometry.  Returns NULL on an invalid mesh and
 * writes a message into err (errlen bytes). */
orc_mesh *orc_mesh_build(int64_t nv, const double *vx, const double *vy,
                         int64_t nc, const int32_t *tri, const double *h,
                         char *err, int errlen);
void orc_mesh_free(orc_mesh *m);
int64_t orc_mesh_ncells(const orc_mesh *m);
int64_t orc_mesh_nedges(const orc_mesh *m);
int64_t orc_mesh_nwalls(const orc_mesh *m);

/* Geometry per cell (nc each) and per local face (3*nc each, face j of cell
 * k at 3k+j).  nbr = -1 marks a wall.  Any pointer may be NULL. */
void orc_mesh_geometry(const orc_mesh *m, double *cx, double *cy,
                       double *area, double *perim, double *len, double *nx,
                       double *ny, double *dx, double *dy, double *wx,
                       double *wy, int32_t *nbr, int32_t *is_left,
                       int32_t *tri_oriented);

/* Reconstruction of one state (Section 2.4).  Outputs (any may be NULL):
 * grad [8*nc]: d/dx,d/dy of eta, Hu, Hv, h; alpha [3*nc]: BJ limiters of
 * eta, Hu, Hv; order [nc]: 2 = second order, 1 = first order;
 * face [15*nc]: per face j the tuple (eta, h, H, u, v) at 15k+5j. */
void orc_reconstruct(const orc_mesh *m, const orc_params *p, const double *H,
                     const double *HU, const double *HV, double *grad,
                     double *alpha, int32_t *order, double *face);

/* Spatial operator R(w) = L(w) of Section 2.3 (per unit area). */
void orc_residual(const orc_mesh *m, const orc_params *p, const double *H,
                  const double *HU, const double *HV, double *RH, double *RHU,
                  double *RHV);

/* Flux of one face, canonical orientation.  left/right = (eta, h, H, u, v)
 * face states; right == NULL means a wall (mirror of left).  Outputs
 * phi[3] (numerical flux per unit length) and p[2] (hydrostatic pressure
 * corrections of the left and right sides). */
void orc_face_flux(const orc_params *p, const double *left,
                   const double *right, double nx, double ny, double *phi,
                   double *pcorr);

/* HLL flux of two conserved states (H, Hu, Hv) across unit normal n, with
 * the wave speeds of Section 2.2 (dry-bed speeds when one side is dry).
 * wl, wr = (H, u, v).  speeds (may be NULL) receives sL, sR, u*, c*
 * (u*, c* are NaN when a side is dry). */
void orc_hll(double g, const double *wl, const double *wr, double nx,
             double ny, double *phi, double *speeds);

/* CFL time step for the state (infinite when no cell is wet). */
double orc_dt(const orc_mesh *m, const orc_params *p, const double *H,
              const double *HU, const double *HV);

/* Advance up to nsteps SSP-RK(2,2) steps from time *t, stopping at t_stop.
 * State arrays are updated in place.  dts (may be NULL) receives the dt of
 * each step.  Returns 0, or -1 on a non-finite state or no valid dt.
 * *clamps counts negative depths set to zero. */
int orc_run(const orc_mesh *m, const orc_params *p, double *H, double *HU,
            double *HV, double *t, int64_t nsteps, double t_stop,
            int64_t *steps_done, double *dts, int64_t *clamps);

/* OpenMP threads of the loops above (default: OMP_NUM_THREADS, else all
 * cores), and the number in use. */
void orc_set_threads(int n);
int orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
