/*
 * c4_oracle.h -- plain FP64 CPU reference of the compact fourth-order
 * staggered-grid scheme for first-order Maxwell's equations
 * (Versano, Turkel, Tsynkov, arXiv 2306.17263).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP path.
 *
 * Layout of every field: a full grid including wall points, row-major with x
 * fastest, index (k*ny + j)*nx + i.  For dim==2 (TM: Ez, Hx, Hy) nz == 1.
 * Component s of E sits at half points along s and at nodes along the other
 * axes; component s of H sits at nodes along s and half points along the
 * others (Section 2, the mesh definitions eq:meshes).  A node axis has N+1
 * points, a half-point axis has N.
 *
 * Errors: functions return 0 on success and a negative value on bad
 * arguments; nothing is printed.
 */
#ifndef C4_ORACLE_H
#define C4_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

enum { OC_EX = 0, OC_EY = 1, OC_EZ = 2, OC_HX = 3, OC_HY = 4, OC_HZ = 5,
       OC_LX = 6, OC_LY = 7, OC_LZ = 8 };               /* L* = h^2 * (Delta E)_s */
enum { OC_CLOSURE_PAPER = 0, OC_CLOSURE_REFLECT = 1 };
enum { OC_LAP_TRACKED = 0, OC_LAP_DISCRETE = 1 };

typedef struct oc_problem oc_problem;

/* Create a cavity problem on [0,1]^dim with n cells per side, CFL number
 * r = h_tau/h, impedance z.  rtol/max_iter control the CG solves of the
 * compact elliptic systems.  Returns NULL on bad arguments. */
oc_problem* oc_create(int dim, int n, double r, double z, int closure,
                      int lap_mode, double rtol, int max_iter);
void oc_destroy(oc_problem* p);

/* Stored extent (nx, ny, nz) of a field, walls included. */
int oc_field_shape(const oc_problem* p, int field, int shape[3]);
int oc_set_field(oc_problem* p, int field, const double* src);
int oc_get_field(const oc_problem* p, int field, double* dst);

/* Advance nsteps full steps (E half-step then H half-step). */
int oc_step(oc_problem* p, long nsteps);
/* Single half-steps with a signed CFL number (negative runs backwards). */
int oc_half_step_e(oc_problem* p, double r_signed);
int oc_half_step_h(oc_problem* p, double r_signed);
/* Taylor start (Section 5.1, eq:talorh, J = 0): with E at tau = 0 and H at
 * tau = 0 set, replace H by H at tau = h_tau/2 (Pade curl for curl E,
 * second-order Laplacian Delta_h for the higher terms). */
int oc_init_h_taylor(oc_problem* p);
/* CG iterations used by the last solve, and the maximum so far. */
int oc_cg_stats(const oc_problem* p, int* last, int* max_seen);

/* Operator-level entry points used by the pins. */
/* Staggered Pade derivative along one line (no 1/h factor): out = A^{-1} D f,
 * n_in inputs, n_in-1 outputs.  node_to_half = 1 when the inputs sit at
 * nodes (outputs at half points), 0 for half points -> interior nodes. */
int oc_pade_line(int n_in, int closure, int node_to_half, const double* f, double* out);
/* y = M x with M = alpha I - beta*L9 on the unknowns of `field`'s grid
 * (alpha = 1 + 2/r^2, beta = r^2/24); x and y are full arrays, wall entries
 * of x must be zero and are written as zero in y. */
int oc_apply_m(const oc_problem* p, int field, const double* x, double* y);
/* Solve M x = b by CG to rtol; returns iterations (>= 0) or < 0 on error. */
int oc_solve_m(const oc_problem* p, int field, const double* b, double* x);
/* RHS of the elliptic system of `field` for the current state, before the
 * solve (the Pade curl of the conditioned source, eq. for Step 1 / Step 2). */
int oc_rhs(const oc_problem* p, int field, double* out);

#ifdef __cplusplus
}
#endif
#endif
