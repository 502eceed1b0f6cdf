/*
 * FP64 CPU reference ("oracle") for the PBD-R solver substep of
 * "Physically Accurate Rigid-Body Dynamics in Particle-Based Simulation"
 * (arXiv 2603.14634).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the GPU library; the two are written independently
 * from the paper and checked against each other.
 *
 * Arrays are structure-of-arrays: a "[3][n]" array stores x components at
 * [0..n), y at [n..2n), z at [2n..3n).  Particles of body b are
 * body_start[b] .. body_start[b+1]-1.
 */
#ifndef PBDR_ORACLE_H
#define PBDR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* flags */
#define ORC_STD_VELOCITY  1u   /* standard PBD velocity V = (X - X_init)/dt (Sec. III-A) */
#define ORC_NO_LIN_MOM    2u   /* drop the linear momentum correction, Eq. (4)  */
#define ORC_NO_ANG_MOM    4u   /* drop the angular momentum correction, Eq. (5) */
#define ORC_PP_AVG_SHIFT  8    /* bits 8-9: pair averaging mode                 */
#define ORC_PP_AVG_MAX    0u   /*   1/max(n_p, n_q)  (default, symmetric)        */
#define ORC_PP_AVG_OWN    1u   /*   1/n_p                                         */
#define ORC_PP_AVG_NONE   2u   /*   plain sum                                     */

typedef struct {
    double h;               /* substep length: Alg. 1's time step */
    double gravity[3];
    double mu;              /* friction coefficient (Tables I, II) */
    double radius;          /* particle radius r; contact distance 2r */
    double search_radius;   /* neighbour predicate radius R_s (<= cell_size) */
    double cell_size;       /* hash-grid cell edge a */
    double grid_origin[3];
    double planes[8][4];    /* half-spaces n.x >= d + r, rows (nx, ny, nz, d), n unit */
    int32_t iterations;     /* solver iterations K */
    int32_t hash_bits;      /* key bits k (6..30) */
    int32_t n_planes;
    int32_t nbr_cap;        /* capacity of each stored neighbour list */
    uint32_t flags;
    int32_t n_threads;      /* OpenMP threads (<= 0: 1) */
} orc_params;

/* Rest pose (Sec. III-C, shape matching): M_b, rest centre of mass, q = x0 - c0. */
void orc_rest_pose(int32_t n, int32_t nb, const int32_t* body_start, const double* mass,
                   const double* x0, double* q_out, double* body_mass_out);

/* FP32 prediction recipe used to place particles in the hash grid. */
void orc_predict32(int32_t n, const orc_params* p, const float* x, const float* v,
                   const float* accel, float* xt_out);

/* Cell key of every particle from FP32 predicted positions. */
void orc_cell_keys(int32_t n, const orc_params* p, const float* xt, uint32_t* key_out);

/* Full index: keys, (key, id)-sorted ids, cell tables, neighbour lists.
 * nbr is [n][nbr_cap] row-major, each row ascending; nbr_count gets the true
 * length (which may exceed nbr_cap; then only nbr_cap entries are stored).
 * Returns the maximum list length. */
int32_t orc_index(int32_t n, const orc_params* p, const int32_t* body, const float* xt,
                  uint32_t* key, uint32_t* sorted_id, uint32_t* cell_start,
                  uint32_t* cell_count, uint32_t* nbr_count, uint32_t* nbr);

/* Rotation part of A (row-major 3x3): the proper rotation maximising tr(R^T A). */
void orc_polar(const double* A, double* R);

/* Symmetric 3x3 pseudo-inverse dropping eigenvalues <= cutoff. */
void orc_pinv_sym3(const double* S, double cutoff, double* out);

/* Momentum conservation constraint, Eqs. (4)-(5), for one body of n particles
 * (AoS [n][3] arrays) of radius r.  Writes the corrected positions and velocities. */
void orc_enforce_momentum(int32_t n, const double* mass, const double* xb, const double* vb,
                          const double* xa, const double* va, double h, double radius, uint32_t flags,
                          double* x_out, double* v_out);

/* One substep (Alg. 1) on the state x, v (SoA [3][n], updated in place).
 * accel may be NULL.  Returns the maximum neighbour-list length. */
int32_t orc_substep(const orc_params* p, int32_t n, int32_t nb, const int32_t* body_start,
                    const double* mass, const double* body_mass, const double* q,
                    const double* accel, double* x, double* v);

/* Per-body state of (x, v) (SoA [3][n]): centre of mass com [nb][3], rotation
 * of shape matching rot9 [nb][9] (row-major, x - c ~ R q), linear momentum
 * P [nb][3] and angular momentum about the centre L [nb][3]. */
void orc_body_state(int32_t n, int32_t nb, const int32_t* body_start, const double* mass, const double* q,
                    const double* x, const double* v, double* com, double* rot9, double* P, double* L);

/* n_substeps consecutive substeps; returns the largest neighbour count seen. */
int32_t orc_run(const orc_params* p, int32_t n, int32_t nb, const int32_t* body_start,
                const double* mass, const double* body_mass, const double* q,
                const double* accel, double* x, double* v, int32_t n_substeps);

#ifdef __cplusplus
}
#endif
#endif
