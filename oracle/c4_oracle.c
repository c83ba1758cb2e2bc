/*
 * c4_oracle.c -- plain FP64 CPU reference of the compact fourth-order
 * staggered (Yee) scheme of Versano, Turkel and Tsynkov (arXiv 2306.17263).
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It is written for a reader holding
 * the paper: every routine is a direct loop over the definitions, with no
 * blocking, fusion or reordering, and cites the passage it follows.
 *
 *   Meshes and wall values ............ Section 2 (eq:meshes, eq:bc_E=0)
 *   Boundary-condition types .......... Section 2.1, Table tab:bc
 *   Ghost values (J = rho = 0) ........ Section 3.3, Corollary cor:ghost_cor
 *   Compact elliptic operator P1 ...... Section 3.2 eq:ell, Definition def:operatorsP
 *   Source conditioning P2 ............ Definition def:operatorsP, Step 1/Step 2
 *   Pade staggered derivative ......... Appendix A.1, eq:lhs
 *   Time stepping (Step 1, Step 2) .... Section 3.4
 *   CG on the SPD systems ............. Section 3.2 and the Conclusions
 *
 * Scaling used throughout (multiply eq:ell by h_tau^2/24 = 1/kappa^2):
 *   M   = (h_tau^2/24) P1 = alpha I - beta L9,   alpha = 1 + 2/r^2, beta = r^2/24,
 *   L9  = h^2 (Delta_h + h^2/6 Upsilon_h)  (dimensionless stencil),
 *   G u = -(h_tau^2/24) P2 u = alpha u + (h^2 Delta_h u)/12,
 *   curl^A = h * curl_h  (the Pade curl without its 1/h).
 * Step 1 then reads  E^{n+1} = E^n + r Phi_E,  M Phi_E = Z curl^A G(H^{n+1/2}),
 * the Laplacian of E is carried along as l = h^2 Delta E:
 *   l^{n+1} = l^n + (24/r^2)(E^{n+1}-E^n) - (24/r) Z curl^A H^{n+1/2},
 * and Step 2 reads  H^{n+3/2} = H^{n+1/2} + r Phi_H,
 *   M Phi_H = -(1/Z) curl^A (alpha E^{n+1} + l^{n+1}/12).
 * In the DISCRETE variant l^{n+1} is replaced by h^2 Delta_h E^{n+1}.
 */
#include "c4_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_CHECK(cond)                                                     \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "c4_oracle: internal check failed: %s (%s:%d)\n",  \
                    #cond, __FILE__, __LINE__);                                \
            abort();                                                           \
        }                                                                      \
    } while (0)

/* One component's grid (eq:meshes).  Along a node axis the stored points are
 * 0..N with the two walls, the unknowns of the elliptic solve are 1..N-1 and
 * the time derivative satisfies a Dirichlet condition.  Along a half-point
 * axis the points are 0..N-1, all unknowns, with a homogeneous Neumann
 * condition realised by the even ghost phi(-1/2) = phi(1/2) (Table tab:bc,
 * Corollary cor:ghost_cor). */
typedef struct {
    int present;
    int half[3];
    int n[3];
    int lo[3], hi[3];
    int active[3];
} comp_t;

struct oc_problem {
    int dim, n, closure, lap_mode, max_iter;
    double r, z, rtol, alpha, beta;
    comp_t comp[6];
    double* f[9];
    int last_it, max_it;
};

static size_t comp_size(const comp_t* c) { return (size_t)c->n[0] * c->n[1] * c->n[2]; }

static size_t ix(const comp_t* c, int i, int j, int k)
{
    return ((size_t)k * c->n[1] + j) * c->n[0] + i;
}

/* Value of grid function a at (i,j,k); an index one or more points outside a
 * half-point axis is mirrored across the wall (even ghost).  Node axes are
 * never left: every stencil is centred on an interior node along them. */
static double at(const comp_t* c, const double* a, int i, int j, int k)
{
    int q[3] = {i, j, k};
    for (int d = 0; d < 3; ++d) {
        if (!c->active[d]) {
            ORACLE_CHECK(q[d] == 0);
            continue;
        }
        if (q[d] < 0 || q[d] >= c->n[d]) {
            ORACLE_CHECK(c->half[d]);
            q[d] = q[d] < 0 ? -1 - q[d] : 2 * c->n[d] - 1 - q[d];
            ORACLE_CHECK(q[d] >= 0 && q[d] < c->n[d]);
        }
    }
    return a[ix(c, q[0], q[1], q[2])];
}

/* h^2 D_ss a at (i,j,k): the standard second difference along axis d
 * (Appendix A.1, matrix D_2). */
static double d2(const comp_t* c, const double* a, int d, int i, int j, int k)
{
    int e[3] = {0, 0, 0};
    e[d] = 1;
    return at(c, a, i - e[0], j - e[1], k - e[2]) - 2.0 * at(c, a, i, j, k) +
           at(c, a, i + e[0], j + e[1], k + e[2]);
}

/* h^4 D_dd D_ee a at (i,j,k), d != e: the second difference along d of the
 * second differences along e. */
static double d2d2(const comp_t* c, const double* a, int d, int e, int i, int j, int k)
{
    static const double w[3] = {1.0, -2.0, 1.0};
    double s = 0.0;
    for (int t = -1; t <= 1; ++t) {
        int q[3] = {i, j, k};
        q[d] += t;
        s += w[t + 1] * d2(c, a, e, q[0], q[1], q[2]);
    }
    return s;
}

static void comp_init(comp_t* c, int dim, int n, int half_axis_mask)
{
    memset(c, 0, sizeof(*c));
    c->present = 1;
    for (int d = 0; d < 3; ++d) {
        c->active[d] = d < dim;
        if (!c->active[d]) {
            c->n[d] = 1;
            c->lo[d] = 0;
            c->hi[d] = 1;
            continue;
        }
        c->half[d] = (half_axis_mask >> d) & 1;
        c->n[d] = c->half[d] ? n : n + 1;
        c->lo[d] = c->half[d] ? 0 : 1;
        c->hi[d] = n;                         /* half: 0..n-1, node: 1..n-1 */
    }
}

static int is_unknown(const comp_t* c, int i, int j, int k)
{
    int q[3] = {i, j, k};
    for (int d = 0; d < 3; ++d)
        if (q[d] < c->lo[d] || q[d] >= c->hi[d]) return 0;
    return 1;
}

static int field_comp(int field) { return field >= OC_LX ? field - OC_LX : field; }

oc_problem* oc_create(int dim, int n, double r, double z, int closure, int lap_mode,
                      double rtol, int max_iter)
{
    if (dim != 2 && dim != 3) return NULL;
    if (n < 8 || !(r > 0.0) || !(z > 0.0) || !(rtol > 0.0) || max_iter < 1) return NULL;
    if (closure != OC_CLOSURE_PAPER && closure != OC_CLOSURE_REFLECT) return NULL;
    if (lap_mode != OC_LAP_TRACKED && lap_mode != OC_LAP_DISCRETE) return NULL;
    oc_problem* p = (oc_problem*)calloc(1, sizeof(oc_problem));
    if (!p) return NULL;
    p->dim = dim;
    p->n = n;
    p->r = r;
    p->z = z;
    p->closure = closure;
    p->lap_mode = lap_mode;
    p->rtol = rtol;
    p->max_iter = max_iter;
    p->alpha = 1.0 + 2.0 / (r * r);   /* kappa^2 h^2 / 12 = 2/r^2 with kappa^2 = 24/h_tau^2 */
    p->beta = r * r / 24.0;
    for (int s = 0; s < 3; ++s) {
        int present = (dim == 3) || (s == 2);   /* TM reduction keeps Ez, Hx, Hy */
        if (present) comp_init(&p->comp[s], dim, n, 1 << s);              /* E_s: half along s */
        int hpresent = (dim == 3) || (s != 2);
        if (hpresent) comp_init(&p->comp[3 + s], dim, n, 7 & ~(1 << s)); /* H_s: node along s */
    }
    for (int f = 0; f < 9; ++f) {
        const comp_t* c = &p->comp[field_comp(f)];
        if (!c->present) continue;
        p->f[f] = (double*)calloc(comp_size(c), sizeof(double));
        if (!p->f[f]) {
            oc_destroy(p);
            return NULL;
        }
    }
    return p;
}

void oc_destroy(oc_problem* p)
{
    if (!p) return;
    for (int f = 0; f < 9; ++f) free(p->f[f]);
    free(p);
}

int oc_field_shape(const oc_problem* p, int field, int shape[3])
{
    if (!p || field < 0 || field > 8 || !p->f[field]) return -1;
    const comp_t* c = &p->comp[field_comp(field)];
    for (int d = 0; d < 3; ++d) shape[d] = c->n[d];
    return 0;
}

/* Tangential E and the carried Laplacian vanish on the walls along E's node
 * axes (eq:bc_E=0 and Table tab:bc_terms: the second time derivative of
 * tangential E is zero there). */
static void zero_node_walls(const comp_t* c, double* a)
{
    for (int k = 0; k < c->n[2]; ++k)
        for (int j = 0; j < c->n[1]; ++j)
            for (int i = 0; i < c->n[0]; ++i) {
                int q[3] = {i, j, k};
                int wall = 0;
                for (int d = 0; d < 3; ++d)
                    if (c->active[d] && !c->half[d] && (q[d] == 0 || q[d] == c->n[d] - 1)) wall = 1;
                if (wall) a[ix(c, i, j, k)] = 0.0;
            }
}

int oc_set_field(oc_problem* p, int field, const double* src)
{
    if (!p || !src || field < 0 || field > 8 || !p->f[field]) return -1;
    const comp_t* c = &p->comp[field_comp(field)];
    memcpy(p->f[field], src, comp_size(c) * sizeof(double));
    if (field <= OC_EZ || field >= OC_LX) zero_node_walls(c, p->f[field]);
    return 0;
}

int oc_get_field(const oc_problem* p, int field, double* dst)
{
    if (!p || !dst || field < 0 || field > 8 || !p->f[field]) return -1;
    const comp_t* c = &p->comp[field_comp(field)];
    memcpy(dst, p->f[field], comp_size(c) * sizeof(double));
    return 0;
}

int oc_cg_stats(const oc_problem* p, int* last, int* max_seen)
{
    if (!p) return -1;
    if (last) *last = p->last_it;
    if (max_seen) *max_seen = p->max_it;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pade staggered first derivative, Appendix A.1 eq:lhs.                     */
/* A f' = D f with D f[m] = f[m+1] - f[m] (the 1/h is left out), A of order  */
/* n_out = n_in - 1: interior rows (1, 22, 1)/24.  Closure rows:            */
/*   PAPER   : (26, -5, 4, -1)/24 and its mirror image, as printed;         */
/*   REFLECT : rows obtained from the image of the line across the wall:    */
/*             outputs at half points see an even derivative, f'(-1/2) =    */
/*             f'(1/2), giving (23, 1)/24; outputs at interior nodes see an */
/*             odd derivative with f'(wall) = 0, giving (22, 1)/24.         */
/* Solved by Gaussian elimination on the band (no pivoting is needed: every */
/* row is strictly diagonally dominant).                                    */
/* ------------------------------------------------------------------------ */
#define BW 3
int oc_pade_line(int n_in, int closure, int node_to_half, const double* f, double* out)
{
    int m = n_in - 1;
    if (!f || !out) return -1;
    if (closure == OC_CLOSURE_PAPER && m < 4) return -1;
    if (m < 2) return -1;
    double* a = (double*)calloc((size_t)m * (2 * BW + 1), sizeof(double)); /* a[row][col-row+BW] */
    double* rhs = (double*)malloc((size_t)m * sizeof(double));
    if (!a || !rhs) {
        free(a);
        free(rhs);
        return -2;
    }
#define A(row, col) a[(size_t)(row) * (2 * BW + 1) + ((col) - (row) + BW)]
    for (int i = 0; i < m; ++i) {
        rhs[i] = f[i + 1] - f[i];
        if (i > 0) A(i, i - 1) = 1.0 / 24.0;
        A(i, i) = 22.0 / 24.0;
        if (i < m - 1) A(i, i + 1) = 1.0 / 24.0;
    }
    if (closure == OC_CLOSURE_PAPER) {
        static const double row0[4] = {26.0, -5.0, 4.0, -1.0};
        for (int t = 0; t < 4; ++t) {
            A(0, t) = row0[t] / 24.0;
            A(m - 1, m - 1 - t) = row0[t] / 24.0;
        }
    } else {
        double corner = node_to_half ? 23.0 : 22.0;
        A(0, 0) = corner / 24.0;
        A(m - 1, m - 1) = corner / 24.0;
    }
    /* forward elimination */
    for (int col = 0; col < m; ++col) {
        double piv = A(col, col);
        for (int row = col + 1; row <= col + BW && row < m; ++row) {
            double l = A(row, col);
            if (l == 0.0) continue;
            l /= piv;
            for (int c2 = col; c2 <= col + BW && c2 < m; ++c2) A(row, c2) -= l * A(col, c2);
            rhs[row] -= l * rhs[col];
        }
    }
    /* back substitution */
    for (int row = m - 1; row >= 0; --row) {
        double s = rhs[row];
        for (int c2 = row + 1; c2 <= row + BW && c2 < m; ++c2) s -= A(row, c2) * out[c2];
        out[row] = s / A(row, row);
    }
#undef A
    free(a);
    free(rhs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Compact elliptic operator, eq:ell scaled by h_tau^2/24:                  */
/*   M phi = alpha phi - beta [ sum_d h^2 D_dd phi                          */
/*                             + (1/6) sum_{d<e} h^4 D_dd D_ee phi ]        */
/* on the unknowns of one component grid; wall entries of phi are zero      */
/* (Dirichlet time derivative), half-axis ghosts are even.                  */
/* ------------------------------------------------------------------------ */
static double l9_at(const comp_t* c, const double* x, int i, int j, int k)
{
    double s = 0.0;
    for (int d = 0; d < 3; ++d)
        if (c->active[d]) s += d2(c, x, d, i, j, k);
    double mixed = 0.0;
    for (int d = 0; d < 3; ++d)
        for (int e = d + 1; e < 3; ++e)
            if (c->active[d] && c->active[e]) mixed += d2d2(c, x, d, e, i, j, k);
    return s + mixed / 6.0;
}

static void apply_m(const oc_problem* p, const comp_t* c, const double* x, double* y)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < c->n[2]; ++k)
        for (int j = 0; j < c->n[1]; ++j)
            for (int i = 0; i < c->n[0]; ++i) {
                size_t q = ix(c, i, j, k);
                y[q] = is_unknown(c, i, j, k) ? p->alpha * x[q] - p->beta * l9_at(c, x, i, j, k) : 0.0;
            }
}

static double dot_unknowns(const comp_t* c, const double* a, const double* b)
{
    double s = 0.0;
    for (int k = c->lo[2]; k < c->hi[2]; ++k)
        for (int j = c->lo[1]; j < c->hi[1]; ++j)
            for (int i = c->lo[0]; i < c->hi[0]; ++i) {
                size_t q = ix(c, i, j, k);
                s += a[q] * b[q];
            }
    return s;
}

/* Conjugate gradients (the solver the paper uses for the SPD systems),
 * started from x = 0, stopped when ||r|| <= rtol ||b|| or after max_iter. */
static int solve_m(const oc_problem* p, const comp_t* c, const double* b, double* x)
{
    size_t sz = comp_size(c);
    double* r = (double*)calloc(sz, sizeof(double));
    double* d = (double*)calloc(sz, sizeof(double));
    double* q = (double*)calloc(sz, sizeof(double));
    if (!r || !d || !q) {
        free(r);
        free(d);
        free(q);
        return -2;
    }
    for (size_t t = 0; t < sz; ++t) x[t] = 0.0;
    for (int kk = c->lo[2]; kk < c->hi[2]; ++kk)
        for (int j = c->lo[1]; j < c->hi[1]; ++j)
            for (int i = c->lo[0]; i < c->hi[0]; ++i) {
                size_t t = ix(c, i, j, kk);
                r[t] = b[t];
                d[t] = b[t];
            }
    double bnorm = sqrt(dot_unknowns(c, b, b));
    double rr = bnorm * bnorm;
    int it = 0;
    while (it < p->max_iter && sqrt(rr) > p->rtol * bnorm) {
        apply_m(p, c, d, q);
        double a = rr / dot_unknowns(c, d, q);
        for (size_t t = 0; t < sz; ++t) {
            x[t] += a * d[t];
            r[t] -= a * q[t];
        }
        double rr_new = dot_unknowns(c, r, r);
        double bet = rr_new / rr;
        for (size_t t = 0; t < sz; ++t) d[t] = r[t] + bet * d[t];
        rr = rr_new;
        ++it;
    }
    free(r);
    free(d);
    free(q);
    return it;
}

/* ------------------------------------------------------------------------ */
/* Sources of the curl.                                                     */
/* ------------------------------------------------------------------------ */
enum { SRC_RAW = 0, SRC_G = 1, SRC_E_RAW = 2 };

/* G u = alpha u + (h^2 Delta_h u)/12 at a point interior along node axes. */
static double g_at(const oc_problem* p, const comp_t* c, const double* u, int i, int j, int k)
{
    double lap = 0.0;
    for (int d = 0; d < 3; ++d)
        if (c->active[d]) lap += d2(c, u, d, i, j, k);
    return p->alpha * u[ix(c, i, j, k)] + lap / 12.0;
}

static int on_node_wall(const comp_t* c, int i, int j, int k)
{
    int q[3] = {i, j, k};
    for (int d = 0; d < 3; ++d)
        if (c->active[d] && !c->half[d] && (q[d] == 0 || q[d] == c->n[d] - 1)) return 1;
    return 0;
}

/* Conditioned E source for Step 2: alpha E + l/12 with the carried l, or,
 * in the DISCRETE variant, alpha E + h^2 Delta_h E / 12.  Both vanish on E's
 * walls. */
static double ge_at(const oc_problem* p, int s, int i, int j, int k)
{
    const comp_t* c = &p->comp[s];
    if (on_node_wall(c, i, j, k)) return 0.0;
    if (p->lap_mode == OC_LAP_TRACKED)
        return p->alpha * p->f[s][ix(c, i, j, k)] + p->f[OC_LX + s][ix(c, i, j, k)] / 12.0;
    return g_at(p, c, p->f[s], i, j, k);
}

/* Value along a curl line of the source component `src`: the conditioned
 * E source (Step 2), raw H (the carried Laplacian) or G(H) (Step 1). */
static double src_value(const oc_problem* p, int src, int kind, int i, int j, int k)
{
    const comp_t* c = &p->comp[src];
    if (src < 3 && kind == SRC_E_RAW) return p->f[src][ix(c, i, j, k)];   /* E itself */
    if (src < 3) return ge_at(p, src, i, j, k);               /* E sources: Step 2 */
    if (kind == SRC_RAW) return p->f[src][ix(c, i, j, k)];    /* H raw */
    return g_at(p, c, p->f[src], i, j, k);                      /* G(H): Step 1 */
}

/* out (target grid, unknown points only) += sign * Pade derivative along
 * axis d of the source component. */
static int add_pade_derivative(const oc_problem* p, int src, int kind, int d, int tgt, double sign,
                               double* out)
{
    const comp_t* cs = &p->comp[src];
    const comp_t* ct = &p->comp[tgt];
    ORACLE_CHECK(cs->half[d] != ct->half[d]);
    int n_in = cs->n[d];
    int n_out = n_in - 1;
    ORACLE_CHECK(n_out == ct->hi[d] - ct->lo[d]);
    int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
    int failed = 0;
    /* Lines are independent; each writes its own outputs. */
#pragma omp parallel for collapse(2) schedule(static) reduction(|| : failed)
    for (int u = ct->lo[a1]; u < ct->hi[a1]; ++u)
        for (int v = ct->lo[a2]; v < ct->hi[a2]; ++v) {
            double* line = (double*)malloc((size_t)n_in * sizeof(double));
            double* der = (double*)malloc((size_t)n_out * sizeof(double));
            if (!line || !der) {
                free(line);
                free(der);
                failed = 1;
                continue;
            }
            int q[3];
            q[a1] = u;
            q[a2] = v;
            for (int t = 0; t < n_in; ++t) {
                q[d] = t;
                line[t] = src_value(p, src, kind, q[0], q[1], q[2]);
            }
            int rc = oc_pade_line(n_in, p->closure, !cs->half[d], line, der);
            ORACLE_CHECK(rc == 0);
            for (int t = 0; t < n_out; ++t) {
                q[d] = ct->lo[d] + t;
                out[ix(ct, q[0], q[1], q[2])] += sign * der[t];
            }
            free(line);
            free(der);
        }
    return failed ? -2 : 0;
}

/* (curl^A V)_s = der_{s+1} V_{s+2} - der_{s+2} V_{s+1}  (curl_h, Section 3.4).
 * Components absent in the TM reduction contribute nothing. */
static int curl_component(const oc_problem* p, int src_base, int kind, int tgt, double scale,
                          double* out)
{
    int s = tgt % 3;
    int s1 = (s + 1) % 3, s2 = (s + 2) % 3;
    const comp_t* ct = &p->comp[tgt];
    memset(out, 0, comp_size(ct) * sizeof(double));
    if (ct->active[s1] && p->comp[src_base + s2].present) {
        int rc = add_pade_derivative(p, src_base + s2, kind, s1, tgt, scale, out);
        if (rc) return rc;
    }
    if (ct->active[s2] && p->comp[src_base + s1].present) {
        int rc = add_pade_derivative(p, src_base + s1, kind, s2, tgt, -scale, out);
        if (rc) return rc;
    }
    return 0;
}

int oc_rhs(const oc_problem* p, int field, double* out)
{
    if (!p || !out || field < 0 || field > 5 || !p->comp[field].present) return -1;
    if (field < 3) return curl_component(p, 3, SRC_G, field, p->z, out);   /* Z curl^A G(H) */
    return curl_component(p, 0, SRC_G, field, -1.0 / p->z, out);           /* -(1/Z) curl^A G_E */
}

int oc_apply_m(const oc_problem* p, int field, const double* x, double* y)
{
    if (!p || !x || !y || field < 0 || field > 5 || !p->comp[field].present) return -1;
    apply_m(p, &p->comp[field], x, y);
    return 0;
}

int oc_solve_m(const oc_problem* p, int field, const double* b, double* x)
{
    if (!p || !b || !x || field < 0 || field > 5 || !p->comp[field].present) return -1;
    return solve_m(p, &p->comp[field], b, x);
}

static void note_iters(oc_problem* p, int it)
{
    p->last_it = it;
    if (it > p->max_it) p->max_it = it;
}

/* Step 1 of Section 3.4 for every E component. */
int oc_half_step_e(oc_problem* p, double rs)
{
    if (!p) return -1;
    for (int s = 0; s < 3; ++s) {
        const comp_t* c = &p->comp[s];
        if (!c->present) continue;
        size_t sz = comp_size(c);
        double* b = (double*)calloc(sz, sizeof(double));
        double* phi = (double*)calloc(sz, sizeof(double));
        double* craw = (double*)calloc(sz, sizeof(double));
        if (!b || !phi || !craw) {
            free(b);
            free(phi);
            free(craw);
            return -2;
        }
        int rc = curl_component(p, 3, SRC_G, s, p->z, b);
        if (!rc && p->lap_mode == OC_LAP_TRACKED) rc = curl_component(p, 3, SRC_RAW, s, 1.0, craw);
        int it = rc ? rc : solve_m(p, c, b, phi);
        if (it < 0) {
            free(b);
            free(phi);
            free(craw);
            return it;
        }
        note_iters(p, it);
        /* The E update of component s reads only H, so components can be
         * updated one after the other. */
        double* e = p->f[s];
        double* l = p->f[OC_LX + s];
        for (int k = c->lo[2]; k < c->hi[2]; ++k)
            for (int j = c->lo[1]; j < c->hi[1]; ++j)
                for (int i = c->lo[0]; i < c->hi[0]; ++i) {
                    size_t q = ix(c, i, j, k);
                    double e_old = e[q];
                    e[q] = e_old + rs * phi[q];
                    if (p->lap_mode == OC_LAP_TRACKED)
                        l[q] += 24.0 / (rs * rs) * (e[q] - e_old) - 24.0 / rs * p->z * craw[q];
                }
        free(b);
        free(phi);
        free(craw);
    }
    return 0;
}

/* Step 2 of Section 3.4 for every H component. */
int oc_half_step_h(oc_problem* p, double rs)
{
    if (!p) return -1;
    for (int s = 3; s < 6; ++s) {
        const comp_t* c = &p->comp[s];
        if (!c->present) continue;
        size_t sz = comp_size(c);
        double* b = (double*)calloc(sz, sizeof(double));
        double* phi = (double*)calloc(sz, sizeof(double));
        if (!b || !phi) {
            free(b);
            free(phi);
            return -2;
        }
        int rc = curl_component(p, 0, SRC_G, s, -1.0 / p->z, b);
        int it = rc ? rc : solve_m(p, c, b, phi);
        if (it < 0) {
            free(b);
            free(phi);
            return it;
        }
        note_iters(p, it);
        double* hh = p->f[s];
        for (int k = c->lo[2]; k < c->hi[2]; ++k)
            for (int j = c->lo[1]; j < c->hi[1]; ++j)
                for (int i = c->lo[0]; i < c->hi[0]; ++i) {
                    size_t q = ix(c, i, j, k);
                    hh[q] += rs * phi[q];
                }
        free(b);
        free(phi);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Taylor start of H (Section 5.1, eq:talorh, J = 0): with H holding H(0)     */
/* and E holding E(0), replace H by                                           */
/*   H(h_tau/2) = H + a H_t + a^2/2 H_tt + a^3/6 H_ttt + a^4/24 H_tttt,      */
/* a = h_tau/2, where (maxh, secondorderh and their derivatives)              */
/*   H_t = -(1/Z) curl E,  H_tt = Delta H,  H_ttt = Delta H_t,               */
/*   H_tttt = Delta H_tt.                                                      */
/* Spatial derivatives: the scheme's Pade curl for curl E, the second-order  */
/* Laplacian Delta_h of Definition def:operatorsP for Delta, with the ghost  */
/* rules of Corollary cor:ghost_cor; on the walls an H component is normal   */
/* to, all its time derivatives vanish (it is constant in time there).       */
/* ------------------------------------------------------------------------ */

/* h^2 Delta_h a at the points of component c off its node walls, 0 on them */
static void lap5(const comp_t* c, const double* a, double* out)
{
    for (int k = 0; k < c->n[2]; ++k)
        for (int j = 0; j < c->n[1]; ++j)
            for (int i = 0; i < c->n[0]; ++i) {
                double v = 0.0;
                if (!on_node_wall(c, i, j, k))
                    for (int d = 0; d < 3; ++d)
                        if (c->active[d]) v += d2(c, a, d, i, j, k);
                out[ix(c, i, j, k)] = v;
            }
}

int oc_init_h_taylor(oc_problem* p)
{
    if (!p) return -1;
    const double r = p->r, z = p->z;
    for (int s = 3; s < 6; ++s) {
        const comp_t* c = &p->comp[s];
        if (!c->present) continue;
        const size_t sz = comp_size(c);
        double* cu = (double*)calloc(sz, sizeof(double));    /* curl^A E = -Z h H_t */
        double* lh = (double*)calloc(sz, sizeof(double));    /* h^2 Delta_h H = h^2 H_tt */
        double* lc = (double*)calloc(sz, sizeof(double));    /* h^2 Delta_h curl^A E */
        double* llh = (double*)calloc(sz, sizeof(double));   /* h^4 Delta_h Delta_h H */
        if (!cu || !lh || !lc || !llh) {
            free(cu); free(lh); free(lc); free(llh);
            return -2;
        }
        int rc = curl_component(p, 0, SRC_E_RAW, s, 1.0, cu);
        if (rc) {
            free(cu); free(lh); free(lc); free(llh);
            return rc;
        }
        /* the curl on the wall points the component is normal to is zero
         * (tangential E vanishes there); curl_component fills the unknowns only */
        lap5(c, p->f[s], lh);
        lap5(c, cu, lc);
        lap5(c, lh, llh);
        /* with a = h_tau/2 = r h/2:  a H_t = -(r/(2Z)) cu,  a^2/2 H_tt = (r^2/8) lh,
         * a^3/6 H_ttt = -(r^3/(48 Z)) lc,  a^4/24 H_tttt = (r^4/384) llh */
        double* hh = p->f[s];
        for (int k = 0; k < c->n[2]; ++k)
            for (int j = 0; j < c->n[1]; ++j)
                for (int i = 0; i < c->n[0]; ++i) {
                    if (on_node_wall(c, i, j, k)) continue;
                    const size_t q = ix(c, i, j, k);
                    hh[q] += -(r / (2.0 * z)) * cu[q] + (r * r / 8.0) * lh[q] - (r * r * r / (48.0 * z)) * lc[q] +
                             (r * r * r * r / 384.0) * llh[q];
                }
        free(cu); free(lh); free(lc); free(llh);
    }
    return 0;
}

int oc_step(oc_problem* p, long nsteps)
{
    if (!p || nsteps < 0) return -1;
    for (long t = 0; t < nsteps; ++t) {
        int rc = oc_half_step_e(p, p->r);
        if (rc) return rc;
        rc = oc_half_step_h(p, p->r);
        if (rc) return rc;
    }
    return 0;
}
