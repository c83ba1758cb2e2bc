// c4m_host.hip -- host runtime behind the C ABI of include/c4m.h:
// configuration checks, workspace carving, the Pade coefficient tables, the
// Chebyshev schedule and the launch sequence of one step.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "c4m_internal.h"
#include "c4m_source.h"

namespace c4m {

// kernels (c4m_kernels_2d.hip, c4m_kernels_3d.hip, c4m_kernels_common.hip)
hipError_t launch_rhs_e_2d(hipStream_t st, bool tracked, const double* hx, const double* hy, double* t0,
                           double* t1, int N, int P, const Coef& cf, const PadeTaps& taps,
                           const PadeLine& line_h2n, double* yb);
bool strip_form_2d(int shape, bool mixed, int sweeps);
hipError_t launch_solve_e_2d(hipStream_t st, int shape, bool mixed, bool tracked, const double* hx, double* ez, double* ge,
                             const double* t0, const double* t1, int N, int P, const Coef& cf,
                             const PadeTaps& taps, const PadeLine& line_h2n, const ChebSchedule& cs, double* yb);
hipError_t launch_rhs_h_2d(hipStream_t st, bool tracked, const double* src, double* t0, double* t1,
                           int N, int P, const Coef& cf, const PadeTaps& taps,
                           const PadeLine& line_n2h, double* yb);
hipError_t launch_solve_h_2d(hipStream_t st, int shape, bool mixed, bool tracked, const double* src, double* hx, double* hy,
                             const double* t1, int N, int P, const Coef& cf, const PadeTaps& taps,
                             const PadeLine& line_n2h, const ChebSchedule& cs, double* yb);
hipError_t launch_pcg_e_2d(hipStream_t st, bool tracked, const double* hx, double* ez, double* ge,
                           const double* t0, double* t1, int N, int P, const Coef& cf, const PadeTaps& taps,
                           const PadeLine& line_h2n, const ChebSchedule& cs, double* const* pt, double* part,
                           PcgState* pst, double rtol, int max_iter);
hipError_t launch_tsolve_e_2d(hipStream_t st, bool tracked, const double* hx, double* ez, double* ge,
                              const double* t0, double* t1, int N, int P, const Coef& cf, const PadeTaps& taps,
                              const PadeLine& line_h2n, const ChebSchedule& cs, double* const* pt,
                              const TransformTables& tt);
hipError_t launch_tsolve_h_2d(hipStream_t st, bool tracked, const double* src, double* hx, double* hy, double* t1,
                              int N, int P, const Coef& cf, const PadeTaps& taps, const PadeLine& line_n2h,
                              const ChebSchedule& cs, double* const* pt, const TransformTables& tt);
hipError_t launch_pcg_h_2d(hipStream_t st, bool tracked, const double* src, double* hx, double* hy, double* t1,
                           int N, int P, const Coef& cf, const PadeTaps& taps, const PadeLine& line_n2h,
                           const ChebSchedule& cs, double* const* pt, double* part, PcgState* pst, double rtol,
                           int max_iter);
hipError_t launch_term3(hipStream_t st, int axis, int mode, const Term3& t, double alpha,
                        const PadeTaps& taps, const PadeLine& L);
hipError_t launch_solve3(hipStream_t st, const Cheb3& c, double* field, double* ge, const double* cur,
                         const Coef& cf, const ChebSchedule& cs);
hipError_t launch_solve3_mixed(hipStream_t st, const Cheb3& c, size_t arr, double* field, double* ge,
                               const double* cur, const Coef& cf, const ChebSchedule& cs);
hipError_t launch_zero_walls(hipStream_t st, double* a, const Box& bx, int P, size_t plane);
hipError_t launch_lap_convert(hipStream_t st, double* a, const double* e, double* out, const Box& bx,
                              int P, size_t plane, double alpha, int mode);
hipError_t launch_count_nonfinite(hipStream_t st, const double* a, const Box& bx, int P,
                                  size_t plane, int* count);
hipError_t launch_nc_e(hipStream_t st, double* ez, const double* hx, const double* hy, int N, int P, double r,
                       double z);
hipError_t launch_nc_h(hipStream_t st, const double* ez, double* hx, double* hy, int N, int P, double r, double z);
hipError_t launch_condition3(hipStream_t st, int mode, const double* src, double* out, const Box& bx, int P,
                             size_t plane, double alpha);
hipError_t launch_taylor_lap(hipStream_t st, const double* a, double* out, const Box& bx, int P, size_t plane);
hipError_t launch_taylor_combine(hipStream_t st, double* h, const double* cu, const double* lh, const Box& bx, int P,
                                 size_t plane, const double c[4]);
hipError_t launch_wall_max(hipStream_t st, const double* a, const Box& bx, int P, size_t plane,
                           unsigned long long* out);
hipError_t launch_put_plane(hipStream_t st, double* a, const double* vals, const Box& bx, int axis, int at,
                            int P, size_t plane);

namespace {

thread_local std::string g_last_error;

c4m_status fail(c4m_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

c4m_status hip_fail(hipError_t e, const char* what)
{
    return fail(C4M_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// Pade tables.  A is the matrix of eq:lhs for one line kind; the rows of
// A^{-1} needed near the two ends are computed exactly from a band LU of A
// (A is strictly diagonally dominant, so no pivoting), the interior row from
// the middle of a long line.  Row m of the folded operator acts on the line
// values f[m-R .. m+R+1]: c_m[u] = W(m, m+u-1) - W(m, m+u), W = A^{-1}
// truncated to |j - m| <= R.
// ---------------------------------------------------------------------------
struct BandLU {
    int n;
    std::vector<double> a;   // [n][7], entry (i, j) at a[i*7 + (j - i + 3)]
    double& at(int i, int j) { return a[(size_t)i * 7 + (j - i + 3)]; }
};

BandLU pade_matrix(int n_out, int closure, bool node_to_half)
{
    BandLU m{n_out, std::vector<double>((size_t)n_out * 7, 0.0)};
    for (int i = 0; i < n_out; ++i) {
        m.at(i, i) = 22.0 / 24.0;
        if (i > 0) m.at(i, i - 1) = 1.0 / 24.0;
        if (i + 1 < n_out) m.at(i, i + 1) = 1.0 / 24.0;
    }
    if (closure == C4M_CLOSURE_PAPER) {
        const double r0[4] = {26.0, -5.0, 4.0, -1.0};
        for (int t = 0; t < 4; ++t) {
            m.at(0, t) = r0[t] / 24.0;
            m.at(n_out - 1, n_out - 1 - t) = r0[t] / 24.0;
        }
    } else {
        const double corner = node_to_half ? 23.0 : 22.0;
        m.at(0, 0) = corner / 24.0;
        m.at(n_out - 1, n_out - 1) = corner / 24.0;
    }
    // in-place LU (Doolittle) on the band
    for (int k = 0; k < n_out; ++k) {
        const double piv = m.at(k, k);
        for (int i = k + 1; i <= std::min(k + 3, n_out - 1); ++i) {
            const double l = m.at(i, k) / piv;
            m.at(i, k) = l;
            if (l == 0.0) continue;
            for (int j = k + 1; j <= std::min(k + 3, n_out - 1); ++j) m.at(i, j) -= l * m.at(k, j);
        }
    }
    return m;
}

// column `col` of A^{-1}
void inverse_column(BandLU& lu, int col, std::vector<double>& x)
{
    const int n = lu.n;
    x.assign(n, 0.0);
    x[col] = 1.0;
    for (int i = 0; i < n; ++i)
        for (int k = std::max(0, i - 3); k < i; ++k) x[i] -= lu.at(i, k) * x[k];
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k <= std::min(i + 3, n - 1); ++k) s -= lu.at(i, k) * x[k];
        x[i] = s / lu.at(i, i);
    }
}

struct PadeHost {
    std::vector<double> rows;   // [n_rows][PADE_TAPS]
    int n_in = 0, n_out = 0, b = 0, all = 0;
    PadeTaps taps{};
};

// W(m, j) for the needed (m, j) pairs, folded into line taps.
PadeHost build_pade(int n_in, int closure, bool node_to_half)
{
    PadeHost ph;
    ph.n_in = n_in;
    ph.n_out = n_in - 1;
    const int n_out = ph.n_out;
    ph.all = n_out <= 2 * PADE_B;
    ph.b = ph.all ? n_out : PADE_B;
    BandLU lu = pade_matrix(n_out, closure, node_to_half);
    std::vector<int> row_ids;
    if (ph.all) {
        for (int m = 0; m < n_out; ++m) row_ids.push_back(m);
    } else {
        for (int m = 0; m < PADE_B; ++m) row_ids.push_back(m);
        for (int m = n_out - PADE_B; m < n_out; ++m) row_ids.push_back(m);
    }
    // columns needed: every j within R of a requested row
    std::vector<std::vector<double>> cols(n_out);
    std::vector<double> tmp;
    auto W = [&](int m, int j) -> double {
        if (j < 0 || j >= n_out || std::abs(j - m) > PADE_R) return 0.0;
        if (cols[j].empty()) {
            inverse_column(lu, j, tmp);
            cols[j] = tmp;
        }
        return cols[j][m];
    };
    ph.rows.assign(row_ids.size() * PADE_TAPS, 0.0);
    for (size_t r = 0; r < row_ids.size(); ++r) {
        const int m = row_ids[r];
        for (int u = -PADE_R; u <= PADE_R + 1; ++u)
            ph.rows[r * PADE_TAPS + (u + PADE_R)] = W(m, m + u - 1) - W(m, m + u);
    }
    // interior taps from the middle row of a long line of the same kind
    const int nl = 4 * PADE_B + 1;
    BandLU lul = pade_matrix(nl, closure, node_to_half);
    const int mid = nl / 2;
    std::vector<double> wrow(2 * PADE_R + 1);
    for (int k = -PADE_R; k <= PADE_R; ++k) {
        inverse_column(lul, mid + k, tmp);
        wrow[k + PADE_R] = tmp[mid];
    }
    auto Wi = [&](int k) { return (k < -PADE_R || k > PADE_R) ? 0.0 : wrow[k + PADE_R]; };
    for (int u = -PADE_R; u <= PADE_R + 1; ++u) ph.taps.c[u + PADE_R] = Wi(u - 1) - Wi(u);
    if (!ph.all) ph.rows.insert(ph.rows.end(), ph.taps.c, ph.taps.c + PADE_TAPS);   // row 2 b
    return ph;
}

// Device image of one line kind: the raw rows, the conditioned rows and the
// interior pair taps, each block starting on a 256-byte boundary.
int pade_table_rows(int n_out) { return n_out <= 2 * PADE_B ? n_out : 2 * PADE_B + 1; }
size_t round32(size_t v) { return (v + 31) & ~(size_t)31; }
size_t line_image_doubles(int n_out)
{
    const size_t rows = (size_t)pade_table_rows(n_out);
    return round32(rows * PADE_TAPS) + round32(rows * COND_TAPS) + round32(PAIR_TAPS);
}

// Conditioned rows: R(m) = sum_u c_m[u] g(m - R + u), where the conditioned
// source g(j) = alpha f(j) + (f(j-1) + f(j+1) - 2 f(j)) / 12 on the line,
// with even ghosts at both ends of a half-point line, zero at the end nodes
// of a node line, and zero off the line.  Folded into taps on f[m-R-1 ..
// m+R+2].  The interior row has no end effects.
std::vector<double> build_line_image(const PadeHost& ph, double alpha, bool half_line)
{
    const int n_out = ph.n_out, n_in = ph.n_in;
    const int rows = pade_table_rows(n_out);
    std::vector<double> img(line_image_doubles(n_out), 0.0);
    std::copy(ph.rows.begin(), ph.rows.end(), img.begin());
    double* crow = img.data() + round32((size_t)rows * PADE_TAPS);
    double* pairs = crow + round32((size_t)rows * COND_TAPS);
    for (int r = 0; r < rows; ++r) {
        const bool interior = !ph.all && r == 2 * ph.b;
        const int m = ph.all || r < ph.b ? r : (interior ? -1 : r - ph.b + (n_out - ph.b));
        const double* c = ph.rows.data() + (size_t)r * PADE_TAPS;
        double* out = crow + (size_t)r * COND_TAPS;
        for (int u = 0; u < PADE_TAPS; ++u) {
            // position j = m - R + u, i.e. window slot u + 1; g(j) uses slots u, u+1, u+2
            double w[3] = {1.0 / 12.0, alpha - 2.0 / 12.0, 1.0 / 12.0};
            if (!interior) {
                const int j = m - PADE_R + u;
                if (j < 0 || j >= n_in) continue;
                if (!half_line && (j == 0 || j == n_in - 1)) continue;
                if (half_line && j == 0) {
                    w[1] += w[0];
                    w[0] = 0.0;
                }
                if (half_line && j == n_in - 1) {
                    w[1] += w[2];
                    w[2] = 0.0;
                }
            }
            for (int v = 0; v < 3; ++v) out[u + v] += c[u] * w[v];
        }
    }
    if (!ph.all) {
        const double* ci = crow + (size_t)(2 * ph.b) * COND_TAPS;
        for (int j = 0; j < COND_TAPS / 2; ++j) pairs[j] = ci[COND_TAPS / 2 - 1 - j];
        for (int j = 0; j < PADE_TAPS / 2; ++j) pairs[COND_TAPS / 2 + j] = ph.taps.c[PADE_TAPS / 2 - 1 - j];
    }
    return img;
}

// ---------------------------------------------------------------------------
// Chebyshev schedule on [alpha, alpha + 16/3 beta] (Saad's Chebyshev
// acceleration); the number of M-applications is the smallest K with
// 1 / T_{K+1}(theta/delta) <= tol.
// ---------------------------------------------------------------------------
ChebSchedule chebyshev(double alpha, double beta, int sweeps, double tol)
{
    ChebSchedule cs{};
    const double lmin = alpha, lmax = alpha + 16.0 / 3.0 * beta;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    if (sweeps <= 0) {
        sweeps = 1;
        while (sweeps < MAX_SWEEPS && 1.0 / cosh((sweeps + 1) * acosh(sigma)) > tol) ++sweeps;
    }
    cs.sweeps = sweeps;
    cs.inv_theta = 1.0 / theta;
    cs.inv_thetaf = (float)cs.inv_theta;
    double rho = 1.0 / sigma;
    for (int k = 0; k < sweeps; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        cs.c1[k] = rn * rho;
        cs.c2[k] = 2.0 * rn / delta;
        cs.c1f[k] = (float)cs.c1[k];
        cs.c2f[k] = (float)cs.c2[k];
        rho = rn;
    }
    return cs;
}

}  // namespace
}  // namespace c4m

using namespace c4m;

// ---------------------------------------------------------------------------
// Problem handle.
// ---------------------------------------------------------------------------
enum { LAP_UNSET = 0, LAP_RAW = 1, LAP_GE = 2 };

// Tangential E (and l) wall values accepted by c4m_set_field: at most this
// fraction of the array's largest magnitude (rounding of sampled data such
// as sin(pi k) at x = 1), stored as exact zeros.
constexpr double C4M_WALL_RTOL = 1e-13;

struct c4m_problem {
    c4m_config cfg{};
    int dim = 0, N = 0, P = 0;
    size_t plane = 0, arr = 0;          // elements per plane / per array
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0, used = 0;
    double* f[6] = {};                  // Ex Ey Ez Hx Hy Hz
    double* ge[3] = {};                 // G_E per E component (carried Laplacian)
    double* tmp[12] = {};
    double* pcg_part = nullptr;         // PCG per-workgroup partial sums
    PcgState* pcg_state = nullptr;      // PCG scalars and statistics
    double* pade_dev[2] = {};           // [0] node->half (n_in N+1), [1] half->node (n_in N)
    double* yband = nullptr;            // 2D strip form: band derivatives near the y-line ends
    double* tr_dev = nullptr;           // transform solver tables
    TransformTables tt{};
    std::vector<double> tr_host;        // their image (kept until the upload completed)
    int* counter = nullptr;
    PadeHost pade_host[2];
    std::vector<double> line_img[2];    // device table images (kept until the upload completed)
    PadeLine line[2]{};
    ChebSchedule cheb{};
    Coef coef{};
    Box box[6]{};
    int lap_state[3] = {LAP_UNSET, LAP_UNSET, LAP_UNSET};
    int64_t steps = 0;
    int nonfinite = 0;
    bool owned_by_batch = false;
    // profiling (C4M_FLAG_PROFILE): event pairs not yet read, and the sums
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    double kernel_ms[C4M_K_COUNT] = {};
    int64_t kernel_launches[C4M_K_COUNT] = {};
    double alg_bytes[C4M_K_COUNT] = {};
    std::map<int64_t, std::pair<hipGraph_t, hipGraphExec_t>> graphs;   // captured runs of steps
    bool direct = false;                // launch steps without graphs (no-allocation call)
    std::vector<Launch3> plan3;         // 3D FP64 Chebyshev step as recorded launches (built on first use)
    std::vector<double> src_cols;       // sourced step: column 0 of A^{-1}, half->node (N-1) then node->half (N)
    void* src_work = nullptr;           // the work buffer that holds them on the device
};

namespace {

bool has_field(int dim, int f)
{
    if (f < 0 || f > 8) return false;
    if (dim == 3) return true;
    return f == C4M_EZ || f == C4M_HX || f == C4M_HY || f == C4M_LZ;
}

int field_comp(int f) { return f >= C4M_LX ? f - C4M_LX : f; }

Box make_box(int dim, int N, int comp)
{
    Box b{};
    const int s = comp % 3;
    const bool is_e = comp < 3;
    for (int d = 0; d < 3; ++d) {
        b.active[d] = d < dim;
        if (!b.active[d]) {
            b.n[d] = 1;
            continue;
        }
        b.half[d] = is_e ? (d == s) : (d != s);
        b.n[d] = b.half[d] ? N : N + 1;
    }
    return b;
}

c4m_status validate(const c4m_config* c)
{
    if (!c) return fail(C4M_EINVAL, "null config");
    if (c->dim != 2 && c->dim != 3) return fail(C4M_EINVAL, "dim must be 2 or 3");
    const int nmax = c->dim == 2 ? 16384 : 1024;
    if (c->n < 8 || c->n > nmax) return fail(C4M_EINVAL, "n out of range");
    if (!(c->cfl > 0.0) || !(c->z > 0.0)) return fail(C4M_EINVAL, "cfl and z must be positive");
    if (c->closure != C4M_CLOSURE_PAPER && c->closure != C4M_CLOSURE_REFLECT)
        return fail(C4M_EINVAL, "bad closure");
    if (c->lap_mode != C4M_LAP_TRACKED && c->lap_mode != C4M_LAP_DISCRETE)
        return fail(C4M_EINVAL, "bad lap_mode");
    if (c->precision != C4M_FP64 && c->precision != C4M_FP32_REFINED)
        return fail(C4M_EINVAL, "bad precision");
    if (c->solver != C4M_SOLVER_CHEBYSHEV && c->solver != C4M_SOLVER_PCG && c->solver != C4M_SOLVER_TRANSFORM)
        return fail(C4M_EINVAL, "bad solver");
    if (c->sweeps < 0 || c->sweeps > MAX_SWEEPS) return fail(C4M_EINVAL, "sweeps out of range");
    if (c->scheme != C4M_SCHEME_C4 && c->scheme != C4M_SCHEME_NC) return fail(C4M_EINVAL, "bad scheme");
    if (c->scheme == C4M_SCHEME_NC) {
        if (c->dim != 2) return fail(C4M_EINVAL, "the NC scheme is 2D");
        if (c->precision != C4M_FP64) return fail(C4M_EINVAL, "the NC scheme runs in FP64");
        // leapfrog with the K4 rows: r^2 (2 (9/8 + 1/24))^2 dim <= 4
        if (!(c->flags & C4M_FLAG_ALLOW_ANY_CFL) && c->cfl > 6.0 / (7.0 * sqrt(2.0)) * (1.0 + 1e-12))
            return fail(C4M_EUNSTABLE, "cfl above the NC stability bound 6/(7 sqrt 2)");
        return C4M_OK;
    }
    if (c->tile_x < 0 || c->tile_x > 4) return fail(C4M_EINVAL, "tile_x (column kernel shape) must be in 0..4");
    if (c->tile_y < 0 || c->tile_y > 8) return fail(C4M_EINVAL, "tile_y (persistent grid multiplier) out of range");
    // Section 4: r <= 1/(sqrt(d) ||A^{-1}||) with ||A^{-1}|| ~ 6/5
    const double bound = 5.0 / (6.0 * sqrt((double)c->dim));
    if (!(c->flags & C4M_FLAG_ALLOW_ANY_CFL) && c->cfl > bound * (1.0 + 1e-12))
        return fail(C4M_EUNSTABLE, "cfl above the stability bound 5/(6 sqrt(dim))");
    if (c->solver == C4M_SOLVER_PCG && c->precision != C4M_FP64)
        return fail(C4M_EINVAL, "the PCG solver runs in FP64 only");
    if (c->solver == C4M_SOLVER_TRANSFORM && c->precision != C4M_FP64)
        return fail(C4M_EINVAL, "the transform solver runs in FP64 only");
    if (c->max_iter < 0 || c->max_iter > 1000) return fail(C4M_EINVAL, "max_iter out of range");
    if (!(c->rtol >= 0.0) || c->rtol >= 1.0) return fail(C4M_EINVAL, "rtol must be in [0, 1)");
    if (c->precision == C4M_FP32_REFINED && (c->sweeps > 3 || (c->dim == 2 && c->tile_x != 0)))
        return fail(C4M_EINVAL, "FP32 refinement: at most 3 sweeps per round and the default tile shape");
    return C4M_OK;
}

struct Layout {
    int P;
    size_t plane, arr, arr_bytes, table_bytes[2], pcg_bytes, band_bytes, tr_bytes, total;
    int n_fields, n_ge, n_tmp;
};

Layout layout(const c4m_config* c)
{
    Layout L{};
    const int N = c->n;
    L.P = (N + 1 + 15) / 16 * 16;
    L.plane = (size_t)(N + 1) * L.P;
    L.arr = c->dim == 2 ? L.plane : L.plane * (N + 1);
    L.arr_bytes = align256(L.arr * sizeof(double));
    L.n_fields = c->dim == 2 ? 3 : 6;
    const bool nc = c->scheme == C4M_SCHEME_NC;
    L.n_ge = (c->lap_mode == C4M_LAP_TRACKED && !nc) ? (c->dim == 2 ? 1 : 3) : 0;
    const bool pcg = c->solver == C4M_SOLVER_PCG && !nc;
    const bool tr = c->solver == C4M_SOLVER_TRANSFORM && !nc;
    // 2D: T0, T1 (+ x, r, two directions, M p, 1/diag, z for PCG);
    // 3D: b, x, d0, d1, curl (+ M p, 1/diag, z for PCG), then the three
    // conditioned sources of the line terms
    L.n_tmp = nc ? 1 : (c->dim == 2 ? (pcg || tr ? 9 : 2) : (pcg ? 8 : 5) + 3);
    L.tr_bytes = tr ? align256(transform_table_doubles(N) * sizeof(double)) : 0;
    L.pcg_bytes = pcg ? align256(3 * ((L.arr + 255) / 256) * sizeof(double)) + 256 : 0;
    for (int k = 0; k < 2; ++k) {
        const int n_out = (k == 0 ? N + 1 : N) - 1;
        L.table_bytes[k] = align256(line_image_doubles(n_out) * sizeof(double));
    }
    // 2D strip form: raw and conditioned derivatives of the band rows at both ends
    L.band_bytes = (c->dim == 2 && !nc) ? align256((size_t)4 * YB_ROWS * L.P * sizeof(double)) : 0;
    L.total = (size_t)(L.n_fields + L.n_ge + L.n_tmp) * L.arr_bytes + L.pcg_bytes + L.band_bytes + L.tr_bytes +
              L.table_bytes[0] + L.table_bytes[1] + 256;
    return L;
}

c4m_status memset_async(c4m_problem* p, void* dst, size_t bytes)
{
    hipError_t e = hipMemsetAsync(dst, 0, bytes, p->stream);
    return e == hipSuccess ? C4M_OK : hip_fail(e, "hipMemsetAsync");
}

// make every E component's G_E array hold G_E
c4m_status ensure_ge(c4m_problem* p)
{
    if (p->cfg.lap_mode != C4M_LAP_TRACKED) return C4M_OK;
    for (int s = 0; s < 3; ++s) {
        if (!p->f[s] || p->lap_state[s] == LAP_GE) continue;
        const int mode = p->lap_state[s] == LAP_RAW ? 0 : 2;
        hipError_t e = launch_lap_convert(p->stream, p->ge[s], p->f[s], nullptr, p->box[s], p->P,
                                          p->plane, p->coef.alpha, mode);
        if (e != hipSuccess) return hip_fail(e, "lap_convert");
        p->lap_state[s] = LAP_GE;
    }
    return C4M_OK;
}

c4m_status copy_field(c4m_problem* p, double* dev, const Box& bx, const double* host_or_dev,
                      bool to_device, bool other_on_device)
{
    const size_t w = (size_t)bx.n[0] * sizeof(double);
    const size_t dpitch = (size_t)p->P * sizeof(double);
    const size_t dense = w * bx.n[1] * bx.n[2];
    // host data pass through a temporary as one contiguous copy; the planes
    // move between the dense and the padded layout on the device
    double* stage = nullptr;
    if (!other_on_device) stage = dev == p->tmp[0] ? p->tmp[1] : p->tmp[0];
    hipError_t e = hipSuccess;
    if (stage && to_device)
        e = hipMemcpyAsync(stage, host_or_dev, dense, hipMemcpyHostToDevice, p->stream);
    const double* other = stage ? stage : host_or_dev;
    const hipMemcpyKind kind = (other_on_device || stage) ? hipMemcpyDeviceToDevice
                                                          : (to_device ? hipMemcpyHostToDevice
                                                                       : hipMemcpyDeviceToHost);
    for (int k = 0; k < bx.n[2] && e == hipSuccess; ++k) {
        double* d = dev + k * p->plane;
        const double* o = other + (size_t)k * bx.n[1] * bx.n[0];
        if (to_device)
            e = hipMemcpy2DAsync(d, dpitch, o, w, w, bx.n[1], kind, p->stream);
        else
            e = hipMemcpy2DAsync((void*)o, w, d, dpitch, w, bx.n[1], kind, p->stream);
    }
    if (e == hipSuccess && stage && !to_device)
        e = hipMemcpyAsync((void*)host_or_dev, stage, dense, hipMemcpyDeviceToHost, p->stream);
    if (e != hipSuccess) return hip_fail(e, "field copy");
    if (!other_on_device) {
        e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    }
    return C4M_OK;
}

c4m_status flush_profile(c4m_problem* p)
{
    if (p->pending.empty()) return C4M_OK;
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (auto& r : p->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            p->kernel_ms[r.cls] += ms;
            p->kernel_launches[r.cls] += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    p->pending.clear();
    return C4M_OK;
}

// Run one launch; with profiling on, bracket it by events on the stream.
template <class F>
c4m_status timed(c4m_problem* p, int cls, const char* what, F&& launch)
{
    const bool prof = (p->cfg.flags & C4M_FLAG_PROFILE) != 0;
    c4m_problem::Rec r{cls, nullptr, nullptr};
    if (prof) {
        if (p->pending.size() >= 4096) {
            c4m_status s = flush_profile(p);
            if (s != C4M_OK) return s;
        }
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess)
            return fail(C4M_EDEVICE, "hipEventCreate");
        if (hipEventRecord(r.a, p->stream) != hipSuccess) return fail(C4M_EDEVICE, "hipEventRecord");
    }
    hipError_t e = launch();
    if (e != hipSuccess) return hip_fail(e, what);
    if (prof) {
        // the stream runs the event, the launches and the event in order:
        // the pair brackets these launches alone; nothing waits here
        if (hipEventRecord(r.b, p->stream) != hipSuccess) return fail(C4M_EDEVICE, "hipEventRecord");
        p->pending.push_back(r);
    }
    return C4M_OK;
}

double pcg_rtol(const c4m_problem* p) { return p->cfg.rtol > 0.0 ? p->cfg.rtol : 1e-14; }
int pcg_max_iter(const c4m_problem* p) { return p->cfg.max_iter > 0 ? p->cfg.max_iter : 16; }

UGrid unknowns(const Box& b)
{
    UGrid g{};
    for (int d = 0; d < 3; ++d) {
        if (!b.active[d]) {
            g.lo[d] = 0;
            g.hi[d] = 1;
            continue;
        }
        g.lo[d] = b.half[d] ? 0 : 1;
        g.hi[d] = b.n[d] - (b.half[d] ? 0 : 1);
        g.neumann[d] = b.half[d];
    }
    return g;
}

// The recorded 3D step of a problem (FP64 Chebyshev form), built once.
const std::vector<Launch3>& problem_plan3(c4m_problem* p)
{
    if (p->plan3.empty()) {
        Plan3In in{};
        for (int c = 0; c < 6; ++c) {
            in.f[c] = p->f[c];
            in.box[c] = p->box[c];
            in.ug[c] = unknowns(p->box[c]);
        }
        for (int c = 0; c < 3; ++c) in.ge[c] = p->ge[c];
        for (int t = 0; t < 8; ++t) in.tmp[t] = p->tmp[t];
        in.P = p->P;
        in.plane = p->plane;
        in.coef = p->coef;
        in.cheb = p->cheb;
        in.line[0] = p->line[0];
        in.line[1] = p->line[1];
        in.tracked = p->cfg.lap_mode == C4M_LAP_TRACKED;
        plan_step3(in, p->plan3);
    }
    return p->plan3;
}

bool plan3_form(const c4m_problem* p)
{
    return p->dim == 3 && p->cfg.scheme == C4M_SCHEME_C4 && p->cfg.solver == C4M_SOLVER_CHEBYSHEV &&
           p->cfg.precision == C4M_FP64;
}

// 3D: Step 1 then Step 2 of Section 3.4, one component at a time.
enum { T3_RAW = 0, T3_G = 1, T3_GE_STORED = 2, T3_GE_DISCRETE = 3 };
constexpr int SRC_G_HOST = T3_G, SRC_GE_DISCRETE_HOST = T3_GE_DISCRETE;
c4m_status step3(c4m_problem* p)
{
    if (plan3_form(p)) {
        // the recorded launches, grouped by class and component for profiling
        const std::vector<Launch3>& rec = problem_plan3(p);
        const PadeTaps taps[2] = {p->pade_host[0].taps, p->pade_host[1].taps};
        c4m_status s = C4M_OK;
        for (size_t i = 0; i < rec.size() && s == C4M_OK;) {
            size_t j = i;
            while (j < rec.size() && rec[j].cls == rec[i].cls && rec[j].group == rec[i].group) ++j;
            s = timed(p, rec[i].cls, "3D step", [&] {
                hipError_t e = hipSuccess;
                for (size_t k = i; k < j && e == hipSuccess; ++k) e = launch3_single(p->stream, rec[k], taps);
                return e;
            });
            i = j;
        }
        return s;
    }
    const bool tracked = p->cfg.lap_mode == C4M_LAP_TRACKED;
    const double z = p->coef.z;
    double *b = p->tmp[0], *x = p->tmp[1], *d0 = p->tmp[2], *d1 = p->tmp[3], *cur = p->tmp[4];
    const bool pcg = p->cfg.solver == C4M_SOLVER_PCG;
    const bool tsolve = p->cfg.solver == C4M_SOLVER_TRANSFORM;
    auto pcg_args = [&](int comp) {
        PcgArgs a{};
        a.x = x;
        a.r = b;
        a.p[0] = d0;
        a.p[1] = d1;
        a.q = p->tmp[5];
        a.dinv = p->tmp[6];
        a.z = p->tmp[7];
        a.part = p->pcg_part;
        a.st = p->pcg_state;
        a.g = unknowns(p->box[comp]);
        a.P = p->P;
        a.plane = p->plane;
        a.alpha = p->coef.alpha;
        a.beta = p->coef.beta;
        a.rtol2 = pcg_rtol(p) * pcg_rtol(p);
        return a;
    };
    c4m_status s = C4M_OK;
    // conditioned sources: G(H_j) for Step 1, G(E_j) on the discrete
    // Laplacian for Step 2 (tracked Step 2 reads the stored G_E)
    double* cond[3] = {p->tmp[pcg ? 8 : 5], p->tmp[pcg ? 9 : 6], p->tmp[pcg ? 10 : 7]};
    auto condition = [&](int first_src, int mode) {
        hipError_t e = hipSuccess;
        for (int j = 0; j < 3 && e == hipSuccess; ++j)
            e = launch_condition3(p->stream, mode, p->f[first_src + j], cond[j], p->box[first_src + j], p->P,
                                  p->plane, p->coef.alpha);
        return e;
    };
    auto term = [&](int axis, int src, const double* sp, int mode, double* out, double scale, int acc, int tgt,
                    int line) {
        Term3 t{sp, out, p->box[src], unknowns(p->box[tgt]), p->P, p->plane, scale, acc};
        return launch_term3(p->stream, axis, mode, t, p->coef.alpha, p->pade_host[line].taps, p->line[line]);
    };
    for (int c = 0; c < 3 && s == C4M_OK; ++c) {
        const int s1 = (c + 1) % 3, s2 = (c + 2) % 3;
        s = timed(p, C4M_K_RHS_E, "rhs E", [&] {
            hipError_t e = c == 0 ? condition(3, SRC_G_HOST) : hipSuccess;
            if (e == hipSuccess) e = term(s1, 3 + s2, cond[s2], T3_RAW, b, z, 0, c, 1);
            if (e == hipSuccess) e = term(s2, 3 + s1, cond[s1], T3_RAW, b, -z, 1, c, 1);
            if (e == hipSuccess && tracked) e = term(s1, 3 + s2, p->f[3 + s2], T3_RAW, cur, 1.0, 0, c, 1);
            if (e == hipSuccess && tracked) e = term(s2, 3 + s1, p->f[3 + s1], T3_RAW, cur, -1.0, 1, c, 1);
            return e;
        });
        if (s != C4M_OK) break;
        s = timed(p, C4M_K_SOLVE_E, "solve E", [&] {
            if (tsolve)
                return launch_transform_solve(p->stream, 3, p->tt, unknowns(p->box[c]), p->P, p->plane, b, x, d0,
                                              p->f[c], tracked ? p->ge[c] : nullptr, cur, p->coef);
            if (pcg)
                return launch_pcg(p->stream, 3, pcg_args(c), pcg_max_iter(p), p->f[c], tracked ? p->ge[c] : nullptr,
                                  cur, p->coef);
            Cheb3 ch{b, x, d0, d1, unknowns(p->box[c]), p->P, p->plane};
            if (p->cfg.precision == C4M_FP32_REFINED)
                return launch_solve3_mixed(p->stream, ch, p->arr, p->f[c], tracked ? p->ge[c] : nullptr, cur,
                                           p->coef, p->cheb);
            return launch_solve3(p->stream, ch, p->f[c], tracked ? p->ge[c] : nullptr, cur, p->coef, p->cheb);
        });
    }
    for (int c = 0; c < 3 && s == C4M_OK; ++c) {
        const int s1 = (c + 1) % 3, s2 = (c + 2) % 3;
        s = timed(p, C4M_K_RHS_H, "rhs H", [&] {
            hipError_t e = (c == 0 && !tracked) ? condition(0, SRC_GE_DISCRETE_HOST) : hipSuccess;
            const double* src1 = tracked ? p->ge[s1] : cond[s1];
            const double* src2 = tracked ? p->ge[s2] : cond[s2];
            if (e == hipSuccess) e = term(s1, s2, src2, T3_RAW, b, -1.0 / z, 0, 3 + c, 0);
            if (e == hipSuccess) e = term(s2, s1, src1, T3_RAW, b, 1.0 / z, 1, 3 + c, 0);
            return e;
        });
        if (s != C4M_OK) break;
        s = timed(p, C4M_K_SOLVE_H, "solve H", [&] {
            if (tsolve)
                return launch_transform_solve(p->stream, 3, p->tt, unknowns(p->box[3 + c]), p->P, p->plane, b, x, d0,
                                              p->f[3 + c], nullptr, nullptr, p->coef);
            if (pcg)
                return launch_pcg(p->stream, 3, pcg_args(3 + c), pcg_max_iter(p), p->f[3 + c], nullptr, nullptr,
                                  p->coef);
            Cheb3 ch{b, x, d0, d1, unknowns(p->box[3 + c]), p->P, p->plane};
            if (p->cfg.precision == C4M_FP32_REFINED)
                return launch_solve3_mixed(p->stream, ch, p->arr, p->f[3 + c], nullptr, nullptr, p->coef, p->cheb);
            return launch_solve3(p->stream, ch, p->f[3 + c], nullptr, nullptr, p->coef, p->cheb);
        });
    }
    return s;
}

// 2D: the strip form's band table (filled by the x-line launches) when the
// configuration runs strips, else nullptr.  One buffer resource spans the
// arrays a strip touches, so the used part of the workspace must stay below
// 4 GiB.
double* band_2d(c4m_problem* p)
{
    return (p->cfg.solver == C4M_SOLVER_CHEBYSHEV && p->yband && p->used < (size_t)0xFFFFF000u &&
            strip_form_2d(p->cfg.tile_x, p->cfg.precision == C4M_FP32_REFINED, p->cheb.sweeps))
               ? p->yband
               : nullptr;
}

// 2D Step 1 (Section 3.4): right-hand side and solve of Ez, with its update.
c4m_status step_e_2d(c4m_problem* p)
{
    const int N = p->N, P = p->P;
    const bool tracked = p->cfg.lap_mode == C4M_LAP_TRACKED;
    double *hx = p->f[C4M_HX], *hy = p->f[C4M_HY], *ez = p->f[C4M_EZ], *ge = p->ge[2];
    double *t0 = p->tmp[0], *t1 = p->tmp[1];
    const bool pcg = p->cfg.solver == C4M_SOLVER_PCG;
    const bool tsolve = p->cfg.solver == C4M_SOLVER_TRANSFORM;
    double* yb = band_2d(p);
    c4m_status s = timed(p, C4M_K_RHS_E, "rhs E", [&] {
        return launch_rhs_e_2d(p->stream, tracked, hx, hy, t0, t1, N, P, p->coef,
                               p->pade_host[1].taps, p->line[1], yb);
    });
    if (s == C4M_OK && tsolve)
        s = timed(p, C4M_K_SOLVE_E, "solve E", [&] {
            return launch_tsolve_e_2d(p->stream, tracked, hx, ez, ge, t0, t1, N, P, p->coef, p->pade_host[1].taps,
                                      p->line[1], p->cheb, p->tmp + 2, p->tt);
        });
    else if (s == C4M_OK && pcg)
        s = timed(p, C4M_K_SOLVE_E, "solve E", [&] {
            return launch_pcg_e_2d(p->stream, tracked, hx, ez, ge, t0, t1, N, P, p->coef, p->pade_host[1].taps,
                                   p->line[1], p->cheb, p->tmp + 2, p->pcg_part, p->pcg_state, pcg_rtol(p),
                                   pcg_max_iter(p));
        });
    else if (s == C4M_OK)
        s = timed(p, C4M_K_SOLVE_E, "solve E", [&] {
            return launch_solve_e_2d(p->stream, p->cfg.tile_x, p->cfg.precision == C4M_FP32_REFINED, tracked, hx, ez, ge, t0, t1, N, P, p->coef,
                                     p->pade_host[1].taps, p->line[1], p->cheb, yb);
        });
    return s;
}

// 2D Step 2 (Section 3.4): right-hand sides and solves of Hx and Hy.
c4m_status step_h_2d(c4m_problem* p)
{
    const int N = p->N, P = p->P;
    const bool tracked = p->cfg.lap_mode == C4M_LAP_TRACKED;
    double *hx = p->f[C4M_HX], *hy = p->f[C4M_HY], *ez = p->f[C4M_EZ], *ge = p->ge[2];
    double *t0 = p->tmp[0], *t1 = p->tmp[1];
    const bool pcg = p->cfg.solver == C4M_SOLVER_PCG;
    const bool tsolve = p->cfg.solver == C4M_SOLVER_TRANSFORM;
    double* yb = band_2d(p);
    c4m_status s = timed(p, C4M_K_RHS_H, "rhs H", [&] {
        return launch_rhs_h_2d(p->stream, tracked, tracked ? ge : ez, t0, t1, N, P, p->coef,
                               p->pade_host[0].taps, p->line[0], yb);
    });
    if (s == C4M_OK && tsolve)
        s = timed(p, C4M_K_SOLVE_H, "solve H", [&] {
            return launch_tsolve_h_2d(p->stream, tracked, tracked ? ge : ez, hx, hy, t1, N, P, p->coef,
                                      p->pade_host[0].taps, p->line[0], p->cheb, p->tmp + 2, p->tt);
        });
    else if (s == C4M_OK && pcg)
        s = timed(p, C4M_K_SOLVE_H, "solve H", [&] {
            return launch_pcg_h_2d(p->stream, tracked, tracked ? ge : ez, hx, hy, t1, N, P, p->coef,
                                   p->pade_host[0].taps, p->line[0], p->cheb, p->tmp + 2, p->pcg_part,
                                   p->pcg_state, pcg_rtol(p), pcg_max_iter(p));
        });
    else if (s == C4M_OK)
        s = timed(p, C4M_K_SOLVE_H, "solve H", [&] {
            return launch_solve_h_2d(p->stream, p->cfg.tile_x, p->cfg.precision == C4M_FP32_REFINED, tracked, tracked ? ge : ez, hx, hy, t1, N, P,
                                     p->coef, p->pade_host[0].taps, p->line[0], p->cheb, yb);
        });
    return s;
}

c4m_status step_once(c4m_problem* p)
{
    const int N = p->N, P = p->P;
    if (p->cfg.scheme == C4M_SCHEME_NC) {
        // the comparison scheme NC (Section 5.2): Yee update with K4 at a = 0
        double *ez = p->f[C4M_EZ], *hx = p->f[C4M_HX], *hy = p->f[C4M_HY];
        c4m_status s = timed(p, C4M_K_STEP_E, "NC E update", [&] {
            return launch_nc_e(p->stream, ez, hx, hy, N, P, p->coef.cfl, p->coef.z);
        });
        if (s == C4M_OK)
            s = timed(p, C4M_K_STEP_H, "NC H update", [&] {
                return launch_nc_h(p->stream, ez, hx, hy, N, P, p->coef.cfl, p->coef.z);
            });
        return s;
    }
    if (p->dim == 2) {
        c4m_status s = step_e_2d(p);
        return s == C4M_OK ? step_h_2d(p) : s;
    }
    return step3(p);
}

// Compulsory FP64 state bytes per launch of each kernel class (temporaries
// excluded): each half-step reads its source field and reads and writes its
// target field (and G_E with the carried Laplacian).
void set_alg_bytes(c4m_problem* p)
{
    // Compulsory FP64 state traffic per launch of each class; each field is
    // counted once per half-step (2D: the x-line kernel of Step 1 reads Hy,
    // the column kernel reads Hx and updates Ez and G_E; 3D: the Step 1
    // right-hand sides read the three H components once, ...).
    const double w = 8.0;
    const bool tracked = p->cfg.lap_mode == C4M_LAP_TRACKED;
    if (p->cfg.scheme == C4M_SCHEME_NC) {
        // E update: Hx, Hy read, Ez read and written; H update: Ez read, Hx, Hy read and written
        const double cells = (double)p->N * p->N;
        p->alg_bytes[C4M_K_STEP_E] = w * cells * 4;
        p->alg_bytes[C4M_K_STEP_H] = w * cells * 5;
        return;
    }
    if (p->dim == 2) {
        const double cells = (double)p->N * p->N;
        p->alg_bytes[C4M_K_RHS_E] = w * cells;
        p->alg_bytes[C4M_K_SOLVE_E] = w * cells * (1 + (tracked ? 4 : 2));
        p->alg_bytes[C4M_K_RHS_H] = w * cells;
        p->alg_bytes[C4M_K_SOLVE_H] = w * cells * 4;
    } else {
        // per launch = per component (three launches of each class a step)
        const double cells = (double)p->N * p->N * p->N;
        p->alg_bytes[C4M_K_RHS_E] = w * cells;                 // one H component's share
        p->alg_bytes[C4M_K_SOLVE_E] = w * cells * (tracked ? 4 : 2);
        p->alg_bytes[C4M_K_RHS_H] = w * cells;
        p->alg_bytes[C4M_K_SOLVE_H] = w * cells * 2;
    }
    p->alg_bytes[C4M_K_STEP_E] = p->alg_bytes[C4M_K_RHS_E] + p->alg_bytes[C4M_K_SOLVE_E];
    p->alg_bytes[C4M_K_STEP_H] = p->alg_bytes[C4M_K_RHS_H] + p->alg_bytes[C4M_K_SOLVE_H];
}

// nsteps steps: runs of up to GRAPH_STEPS steps are captured once each as a
// HIP graph and replayed; launches go to the stream directly when the
// launches are profiled, the stream is the null stream (which cannot be
// captured) or the caller is capturing the stream already.
constexpr int64_t GRAPH_STEPS = 32;

// The graph of a run of len steps, captured on the problem's stream the
// first time it is asked for (nothing runs: capture only records).
c4m_status step_graph(c4m_problem* p, int64_t len, hipGraphExec_t* out)
{
    auto it = p->graphs.find(len);
    if (it == p->graphs.end()) {
        hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        c4m_status s = C4M_OK;
        for (int64_t t = 0; t < len && s == C4M_OK; ++t) s = step_once(p);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(p->stream, &g);
        if (s != C4M_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        it = p->graphs.emplace(len, std::make_pair(g, x)).first;
    }
    *out = it->second.second;
    return C4M_OK;
}

// Whether c4m_step launches the steps directly rather than as graphs.
bool steps_direct(c4m_problem* p)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    bool direct = (p->cfg.flags & (C4M_FLAG_PROFILE | C4M_FLAG_DIRECT)) || !p->stream || p->direct;
    if (!direct && hipStreamIsCapturing(p->stream, &cap) != hipSuccess) direct = true;
    return direct || cap != hipStreamCaptureStatusNone;
}

c4m_status run_steps(c4m_problem* p, int64_t nsteps)
{
    if (steps_direct(p)) {
        for (int64_t t = 0; t < nsteps; ++t) {
            c4m_status s = step_once(p);
            if (s != C4M_OK) return s;
            ++p->steps;
        }
        return C4M_OK;
    }
    int64_t left = nsteps;
    while (left > 0) {
        const int64_t len = std::min(left, GRAPH_STEPS);
        hipGraphExec_t x = nullptr;
        c4m_status s = step_graph(p, len, &x);
        if (s != C4M_OK) return s;
        hipError_t e = hipGraphLaunch(x, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        left -= len;
        p->steps += len;
    }
    return C4M_OK;
}

void drop_graphs(c4m_problem* p)
{
    for (auto& kv : p->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    p->graphs.clear();
}

}  // namespace

extern "C" {

const char* c4m_status_string(c4m_status s)
{
    switch (s) {
        case C4M_OK: return "ok";
        case C4M_EINVAL: return "invalid argument";
        case C4M_ENOMEM: return "workspace too small";
        case C4M_EDEVICE: return "device error";
        case C4M_ESTATE: return "invalid state";
        case C4M_ENOCONV: return "solver did not converge";
        case C4M_EUNSTABLE: return "cfl above the stability bound";
        case C4M_ENONFINITE: return "non-finite value";
    }
    return "unknown status";
}

const char* c4m_last_error(void) { return g_last_error.c_str(); }

c4m_status c4m_config_default(c4m_config* cfg)
{
    if (!cfg) return fail(C4M_EINVAL, "null config");
    memset(cfg, 0, sizeof(*cfg));
    cfg->dim = 2;
    cfg->n = 64;
    cfg->cfl = 0.5;
    cfg->z = 1.0;
    cfg->closure = C4M_CLOSURE_PAPER;
    cfg->lap_mode = C4M_LAP_TRACKED;
    cfg->precision = C4M_FP64;
    cfg->solver = C4M_SOLVER_CHEBYSHEV;
    return C4M_OK;
}

c4m_status c4m_workspace_bytes(const c4m_config* cfg, size_t* bytes)
{
    c4m_status s = validate(cfg);
    if (s != C4M_OK) return s;
    if (!bytes) return fail(C4M_EINVAL, "null bytes");
    *bytes = layout(cfg).total;
    return C4M_OK;
}

c4m_status c4m_create(const c4m_config* cfg_in, void* d_workspace, size_t bytes, void* hip_stream,
                      c4m_problem** out)
{
    c4m_status s = validate(cfg_in);
    if (s != C4M_OK) return s;
    // the NC scheme carries no Laplacian of E
    c4m_config cfg_local = *cfg_in;
    if (cfg_local.scheme == C4M_SCHEME_NC) cfg_local.lap_mode = C4M_LAP_DISCRETE;
    const c4m_config* cfg = &cfg_local;
    if (!out) return fail(C4M_EINVAL, "null out");
    *out = nullptr;
    if (!d_workspace || ((uintptr_t)d_workspace & 255)) return fail(C4M_EINVAL, "workspace must be 256-byte aligned");
    const Layout L = layout(cfg);
    if (bytes < L.total) return fail(C4M_ENOMEM, "workspace smaller than c4m_workspace_bytes");
    c4m_problem* p = new (std::nothrow) c4m_problem();
    if (!p) return fail(C4M_ENOMEM, "host allocation");
    p->cfg = *cfg;
    p->dim = cfg->dim;
    p->N = cfg->n;
    p->P = L.P;
    p->plane = L.plane;
    p->arr = L.arr;
    p->stream = (hipStream_t)hip_stream;
    p->ws = (char*)d_workspace;
    p->ws_bytes = bytes;
    char* cur = p->ws;
    auto take = [&](size_t nbytes) {
        char* r = cur;
        cur += nbytes;
        return r;
    };
    for (int c = 0; c < 6; ++c)
        if (has_field(p->dim, c)) {
            p->f[c] = (double*)take(L.arr_bytes);
            p->box[c] = make_box(p->dim, p->N, c);
        }
    if (cfg->lap_mode == C4M_LAP_TRACKED)
        for (int c = 0; c < 3; ++c)
            if (p->f[c]) p->ge[c] = (double*)take(L.arr_bytes);
    for (int t = 0; t < L.n_tmp; ++t) p->tmp[t] = (double*)take(L.arr_bytes);
    if (L.pcg_bytes) {
        p->pcg_state = (PcgState*)take(256);
        p->pcg_part = (double*)take(L.pcg_bytes - 256);
    }
    if (L.band_bytes) p->yband = (double*)take(L.band_bytes);
    if (L.tr_bytes) p->tr_dev = (double*)take(L.tr_bytes);
    p->pade_dev[0] = (double*)take(L.table_bytes[0]);
    p->pade_dev[1] = (double*)take(L.table_bytes[1]);
    p->counter = (int*)take(256);
    p->used = (size_t)(cur - p->ws);

    const double r = cfg->cfl;
    p->coef.alpha = 1.0 + 2.0 / (r * r);
    p->coef.beta = r * r / 24.0;
    p->coef.cfl = r;
    p->coef.z = cfg->z;
    p->coef.ge_gain = 1.0 + 4.0 / (r * r);
    p->coef.ge_curl = 2.0 / r * cfg->z;
    if (cfg->precision == C4M_FP32_REFINED) {
        // two FP32 rounds of s applications around one FP64 residual; the
        // tile halo (and ChebSchedule::sweeps) is 2 s + 1
        const int s_round = cfg->sweeps > 0 ? cfg->sweeps : 2;
        p->cheb = chebyshev(p->coef.alpha, p->coef.beta, 2 * s_round + 1, CHEB_TOL);
        p->cheb.sweeps = 2 * s_round + 1;
    } else {
        p->cheb = chebyshev(p->coef.alpha, p->coef.beta, cfg->sweeps, CHEB_TOL);
    }
    set_alg_bytes(p);

    for (int k = 0; k < 2; ++k) {
        const int n_in = k == 0 ? p->N + 1 : p->N;
        p->pade_host[k] = build_pade(n_in, cfg->closure, k == 0);
        const PadeHost& ph = p->pade_host[k];
        // line 1 (Step 1 y-lines of Hx) runs over half points, line 0 over nodes
        p->line_img[k] = build_line_image(ph, p->coef.alpha, k == 1);
        const int rows = pade_table_rows(ph.n_out);
        const double* crows = p->pade_dev[k] + round32((size_t)rows * PADE_TAPS);
        const double* pairs = crows + round32((size_t)rows * COND_TAPS);
        p->line[k] = PadeLine{p->pade_dev[k], ph.n_in, ph.n_out, ph.b, ph.all, crows, pairs};
        hipError_t e = hipMemcpyAsync(p->pade_dev[k], p->line_img[k].data(), p->line_img[k].size() * sizeof(double),
                                      hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) {
            delete p;
            return hip_fail(e, "table upload");
        }
    }
    if (p->tr_dev) {
        p->tr_host.resize(transform_table_doubles(p->N));
        build_transform_tables(p->N, p->tr_host.data(), &p->tt, p->tr_dev);
        hipError_t e = hipMemcpyAsync(p->tr_dev, p->tr_host.data(), p->tr_host.size() * sizeof(double),
                                      hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) {
            delete p;
            return hip_fail(e, "transform table upload");
        }
    }
    // zero fields, G_E and temporaries
    const size_t zero_bytes = (size_t)((char*)(p->tr_dev ? p->tr_dev : p->pade_dev[0]) - p->ws);
    s = memset_async(p, p->ws, zero_bytes);
    if (s == C4M_OK) s = memset_async(p, p->counter, 256);
    if (s == C4M_OK) {
        hipError_t e = hipStreamSynchronize(p->stream);   // host tables may be released after this
        if (e != hipSuccess) s = hip_fail(e, "hipStreamSynchronize");
    }
    if (s != C4M_OK) {
        delete p;
        return s;
    }
    *out = p;
    return C4M_OK;
}

c4m_status c4m_field_shape(const c4m_problem* p, c4m_field f, int64_t shape[3])
{
    if (!p || !shape || !has_field(p->dim, f)) return fail(C4M_EINVAL, "bad field");
    const Box& b = p->box[field_comp(f)];
    shape[0] = b.n[2];
    shape[1] = b.n[1];
    shape[2] = b.n[0];
    return C4M_OK;
}

c4m_status c4m_set_field(c4m_problem* p, c4m_field f, const double* src, int src_on_device)
{
    if (!p || !src || !has_field(p->dim, f)) return fail(C4M_EINVAL, "bad field");
    const int c = field_comp(f);
    const bool is_lap = f >= C4M_LX;
    if (is_lap && p->cfg.lap_mode != C4M_LAP_TRACKED) return C4M_OK;   // recomputed each step
    const Box& bx = p->box[c];
    if (c < 3) {
        // Tangential E and l vanish on the PEC walls (eq:bc_E=0): reject
        // wall values above rounding of the array's scale, before anything
        // changes.  Host data are checked here, device data in a staging
        // copy in the first temporary.
        double all = 0.0, wall = 0.0;
        if (!src_on_device) {
            const size_t nx = bx.n[0], ny = bx.n[1], nz = bx.n[2];
            for (size_t k = 0; k < nz; ++k)
                for (size_t j = 0; j < ny; ++j)
                    for (size_t i = 0; i < nx; ++i) {
                        double v = fabs(src[(k * ny + j) * nx + i]);
                        if (v != v) v = INFINITY;
                        all = v > all ? v : all;
                        const size_t q[3] = {i, j, k};
                        bool w = false;
                        for (int d = 0; d < 3; ++d)
                            w = w || (bx.active[d] && !bx.half[d] && (q[d] == 0 || q[d] == (size_t)bx.n[d] - 1));
                        if (w) wall = v > wall ? v : wall;
                    }
        } else {
            c4m_status s = copy_field(p, p->tmp[0], bx, src, true, true);
            if (s != C4M_OK) return s;
            unsigned long long* mx = (unsigned long long*)((char*)p->counter + 64);
            unsigned long long h[2] = {0, 0};
            hipError_t e = hipMemsetAsync(mx, 0, 2 * sizeof(unsigned long long), p->stream);
            if (e == hipSuccess) e = launch_wall_max(p->stream, p->tmp[0], bx, p->P, p->plane, mx);
            if (e == hipSuccess) e = hipMemcpyAsync(h, mx, sizeof(h), hipMemcpyDeviceToHost, p->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
            if (e != hipSuccess) return hip_fail(e, "wall check");
            memcpy(&all, &h[0], sizeof(double));
            memcpy(&wall, &h[1], sizeof(double));
        }
        if (!(wall <= C4M_WALL_RTOL * all))
            return fail(C4M_EINVAL, "tangential E (and l) must vanish on the PEC walls");
    }
    if (!is_lap && c < 3 && p->cfg.lap_mode == C4M_LAP_TRACKED && p->lap_state[c] == LAP_GE) {
        // keep l: convert G_E back to l with the old E before E changes
        hipError_t e = launch_lap_convert(p->stream, p->ge[c], p->f[c], p->ge[c], bx, p->P,
                                          p->plane, p->coef.alpha, 1);
        if (e != hipSuccess) return hip_fail(e, "lap_convert");
        p->lap_state[c] = LAP_RAW;
    }
    double* dst = is_lap ? p->ge[c] : p->f[c];
    c4m_status s = copy_field(p, dst, bx, src, true, src_on_device != 0);
    if (s != C4M_OK) return s;
    if (c < 3) {
        // values at rounding level become exact zeros
        hipError_t e = launch_zero_walls(p->stream, dst, bx, p->P, p->plane);
        if (e != hipSuccess) return hip_fail(e, "zero_walls");
    }
    if (is_lap) p->lap_state[c] = LAP_RAW;
    return C4M_OK;
}

c4m_status c4m_set_boundary(c4m_problem* p, c4m_field f, int32_t face, const double* vals, int vals_on_device)
{
    if (!p || !vals || !has_field(p->dim, f)) return fail(C4M_EINVAL, "bad field");
    if (face < 0 || face >= 2 * p->dim) return fail(C4M_EINVAL, "face must be 2 axis + side with axis < dim");
    const int axis = face / 2, side = face % 2;
    const int c = field_comp(f);
    const Box& bx = p->box[c];
    const size_t count = (size_t)bx.n[0] * bx.n[1] * bx.n[2] / bx.n[axis];
    if (c < 3) {
        // E_s and l_s: points on the walls normal to the other axes only,
        // where they must vanish (eq:bc_E=0)
        if (axis == c) return fail(C4M_EINVAL, "E_s has no points on the walls normal to axis s");
        std::vector<double> h(count);
        const double* hv = vals;
        if (vals_on_device) {
            hipError_t e = hipMemcpyAsync(h.data(), vals, count * sizeof(double), hipMemcpyDeviceToHost, p->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
            if (e != hipSuccess) return hip_fail(e, "boundary copy");
            hv = h.data();
        }
        for (size_t i = 0; i < count; ++i)
            if (hv[i] != 0.0) return fail(C4M_EINVAL, "tangential E (and l) must vanish on the PEC walls");
        return C4M_OK;
    }
    // H_s: points on the two walls normal to axis s, where it keeps its
    // value for all time (eq:BC_H)
    if (axis != c - 3) return fail(C4M_EINVAL, "H_s has points only on the walls normal to axis s");
    const double* dv = vals;
    if (!vals_on_device) {
        hipError_t e = hipMemcpyAsync(p->tmp[0], vals, count * sizeof(double), hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) return hip_fail(e, "boundary copy");
        dv = p->tmp[0];
    }
    hipError_t e = launch_put_plane(p->stream, p->f[c], dv, bx, axis, side ? bx.n[axis] - 1 : 0, p->P, p->plane);
    if (e == hipSuccess && !vals_on_device) e = hipStreamSynchronize(p->stream);
    return e == hipSuccess ? C4M_OK : hip_fail(e, "set_boundary");
}

c4m_status c4m_get_field(c4m_problem* p, c4m_field f, double* dst, int dst_on_device)
{
    if (!p || !dst || !has_field(p->dim, f)) return fail(C4M_EINVAL, "bad field");
    const int c = field_comp(f);
    const bool is_lap = f >= C4M_LX;
    const double* srcp = p->f[c];
    if (is_lap) {
        if (p->cfg.lap_mode != C4M_LAP_TRACKED || p->lap_state[c] == LAP_UNSET) {
            // l = L5 E, produced in a temporary (as G_E, then converted)
            hipError_t e = launch_lap_convert(p->stream, p->tmp[0], p->f[c], nullptr, p->box[c], p->P,
                                              p->plane, p->coef.alpha, 2);
            if (e == hipSuccess)
                e = launch_lap_convert(p->stream, p->tmp[0], p->f[c], p->tmp[0], p->box[c], p->P,
                                       p->plane, p->coef.alpha, 1);
            if (e != hipSuccess) return hip_fail(e, "lap_convert");
            srcp = p->tmp[0];
        } else if (p->lap_state[c] == LAP_GE) {
            hipError_t e = launch_lap_convert(p->stream, p->ge[c], p->f[c], p->tmp[0], p->box[c], p->P,
                                              p->plane, p->coef.alpha, 1);
            if (e != hipSuccess) return hip_fail(e, "lap_convert");
            srcp = p->tmp[0];
        } else {
            srcp = p->ge[c];
        }
    }
    return copy_field(p, (double*)srcp, p->box[c], dst, false, dst_on_device != 0);
}

// With C4M_FLAG_CHECK_FINITE: scan the fields for NaN / Inf, wait, and
// report ENONFINITE (sticky in c4m_info).
static c4m_status finite_check(c4m_problem* p)
{
    if (!(p->cfg.flags & C4M_FLAG_CHECK_FINITE)) return C4M_OK;
    hipError_t e = hipMemsetAsync(p->counter, 0, sizeof(int), p->stream);
    for (int c = 0; c < 6 && e == hipSuccess; ++c)
        if (p->f[c]) e = launch_count_nonfinite(p->stream, p->f[c], p->box[c], p->P, p->plane, p->counter);
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, p->counter, sizeof(int), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "finite check");
    if (h) {
        p->nonfinite = 1;
        return fail(C4M_ENONFINITE, "non-finite field values");
    }
    return C4M_OK;
}

c4m_status c4m_step(c4m_problem* p, int64_t nsteps)
{
    if (!p || nsteps < 0) return fail(C4M_EINVAL, "bad step count");
    if (nsteps == 0) return C4M_OK;
    c4m_status s = ensure_ge(p);
    if (s != C4M_OK) return s;
    s = run_steps(p, nsteps);
    if (s != C4M_OK) return s;
    return finite_check(p);
}

c4m_status c4m_prepare(c4m_problem* p, int64_t nsteps)
{
    if (!p || nsteps < 0) return fail(C4M_EINVAL, "bad step count");
    if (nsteps == 0 || steps_direct(p)) return C4M_OK;
    const int64_t full = std::min(nsteps, GRAPH_STEPS), rest = nsteps % GRAPH_STEPS;
    hipGraphExec_t x = nullptr;
    c4m_status s = step_graph(p, full, &x);
    if (s == C4M_OK && rest != 0 && nsteps > GRAPH_STEPS) s = step_graph(p, rest, &x);
    return s;
}

c4m_status c4m_set_stream(c4m_problem* p, void* stream)
{
    if (!p) return fail(C4M_EINVAL, "null problem");
    if (p->owned_by_batch) return fail(C4M_ESTATE, "problem belongs to a batch");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    p->stream = (hipStream_t)stream;
    return C4M_OK;
}

c4m_status c4m_init_h_taylor(c4m_problem* p)
{
    if (!p) return fail(C4M_EINVAL, "null problem");
    if (p->cfg.scheme != C4M_SCHEME_C4) return fail(C4M_EINVAL, "the Taylor start belongs to the compact scheme");
    if (p->steps != 0) return fail(C4M_ESTATE, "the Taylor start takes the fields at tau = 0 (no step taken)");
    const double r = p->cfg.cfl, z = p->cfg.z;
    // a = h_tau/2 = r h/2:  a H_t = -(r/(2Z)) curl^A E,  a^2/2 H_tt = (r^2/8) L5 H,
    // a^3/6 H_ttt = -(r^3/(48 Z)) L5 curl^A E,  a^4/24 H_tttt = (r^4/384) L5 L5 H
    const double c[4] = {-r / (2.0 * z), r * r / 8.0, -r * r * r / (48.0 * z), r * r * r * r / 384.0};
    double *cu = p->tmp[0], *lh = p->tmp[1];
    for (int comp = 0; comp < 3; ++comp) {
        double* h = p->f[3 + comp];
        if (!h) continue;
        const Box& bh = p->box[3 + comp];
        hipError_t e = hipMemsetAsync(cu, 0, p->arr * sizeof(double), p->stream);
        // (curl^A E)_c = delta_{c1} E_{c2} - delta_{c2} E_{c1}: every E
        // derivative runs along a node axis of E (a node -> half line)
        int first = 1;
        for (int t = 0; t < 2 && e == hipSuccess; ++t) {
            const int axis = t == 0 ? (comp + 1) % 3 : (comp + 2) % 3;
            const int src = t == 0 ? (comp + 2) % 3 : (comp + 1) % 3;
            if (axis >= p->dim || !p->f[src]) continue;
            Term3 tm{p->f[src], cu, p->box[src], unknowns(bh), p->P, p->plane, t == 0 ? 1.0 : -1.0, first ? 0 : 1};
            e = launch_term3(p->stream, axis, T3_RAW, tm, p->coef.alpha, p->pade_host[0].taps, p->line[0]);
            first = 0;
        }
        if (e == hipSuccess) e = launch_taylor_lap(p->stream, h, lh, bh, p->P, p->plane);
        if (e == hipSuccess) e = launch_taylor_combine(p->stream, h, cu, lh, bh, p->P, p->plane, c);
        if (e != hipSuccess) return hip_fail(e, "Taylor start");
    }
    return C4M_OK;
}

// ---------------------------------------------------------------------------
// Sources (2D TM): the step of c4m_step with the correction of each
// half-step's right-hand side for J (c4m_source.hip).
// ---------------------------------------------------------------------------
static bool takes_sources(const c4m_problem* p)
{
    return p && p->dim == 2 && p->cfg.scheme == C4M_SCHEME_C4 && p->cfg.closure == C4M_CLOSURE_PAPER;
}

// the two Pade columns of the correction's right-hand sides
static size_t src_work_bytes(const c4m_problem* p)
{
    return ((size_t)(2 * p->N - 1) * sizeof(double) + 255) & ~(size_t)255;
}

static ChebGeom src_geom(const c4m_problem* p, int comp)
{
    const Box& bx = p->box[comp];
    ChebGeom g{};
    for (int d = 0; d < 2; ++d) {
        g.n[d] = bx.n[d];
        g.half[d] = bx.half[d];
        g.lo[d] = bx.half[d] ? 0 : 1;
        g.hi[d] = bx.half[d] ? bx.n[d] - 1 : bx.n[d] - 2;
    }
    g.P = p->P;
    g.alpha = p->coef.alpha;
    g.beta = p->coef.beta;
    return g;
}

size_t c4m_source_work_bytes(const c4m_problem* p)
{
    return takes_sources(p) ? src_work_bytes(p) : 0;
}

c4m_status c4m_step_source(c4m_problem* p, const c4m_source_tm* src, void* work, size_t work_bytes)
{
    if (!p || !src) return fail(C4M_EINVAL, "null argument");
    if (p->owned_by_batch) return fail(C4M_ESTATE, "problem belongs to a batch");
    if (!takes_sources(p)) return fail(C4M_EINVAL, "sources take a 2D problem of the compact scheme with the PAPER closure");
    if (!work || work_bytes < src_work_bytes(p) || ((uintptr_t)work & 255))
        return fail(C4M_EINVAL, "work buffer too small or not 256-byte aligned");
    const int N = p->N;
    if (p->src_cols.empty()) {
        // column 0 of A^{-1} for the two line kinds of the 2D curl (eq:lhs)
        std::vector<double> col;
        BandLU a = pade_matrix(N - 1, C4M_CLOSURE_PAPER, false);
        inverse_column(a, 0, col);
        p->src_cols = col;
        BandLU c = pade_matrix(N, C4M_CLOSURE_PAPER, true);
        inverse_column(c, 0, col);
        p->src_cols.insert(p->src_cols.end(), col.begin(), col.end());
    }
    double* wc = (double*)work;
    double* vc = wc + (N - 1);
    if (work != p->src_work) {
        // the tables go to a work buffer once; later calls with it find them there
        hipError_t e = hipMemcpyAsync(wc, p->src_cols.data(), p->src_cols.size() * sizeof(double),
                                      hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) return hip_fail(e, "source tables");
        p->src_work = work;
    }
    c4m_status s = ensure_ge(p);
    if (s != C4M_OK) return s;
    const double r = p->cfg.cfl, z = p->cfg.z, h = 1.0 / N;
    const bool tracked = p->cfg.lap_mode == C4M_LAP_TRACKED;
    auto group = [&](int f) {
        SrcTile a{};
        a.s = *src;
        a.cols = f == C4M_EZ ? wc : vc;
        a.c = SrcCoef{h, (r * h) * (r * h) / 24.0, h * h / 24.0, p->coef.alpha, p->coef.beta, z};
        a.g = src_geom(p, f);
        a.u = SrcUpdate{p->f[f], nullptr, nullptr, nullptr, r, z, a.c.ht2, 0.0, 0.0};
        if (f == C4M_EZ && tracked) {
            a.u.ge = p->ge[2];
            a.u.jz = src->jz;
            a.u.jz_tt = src->jz_tt;
            a.u.ge_gain = p->coef.ge_gain;
            a.u.ge_src = 2.0 / r * h;
        }
        a.comp = f == C4M_EZ ? 2 : f - C4M_HX;
        a.N = N;
        a.K = p->cheb.sweeps;
        return launch_src_group(p->stream, a);
    };
    // Compulsory bytes of one correction group (its source arrays read once,
    // the field, and G_E with the carried Laplacian, read and written),
    // averaged over the three groups of a step: the E group reads four
    // arrays, each H group two.
    const double cells = (double)N * N;
    p->alg_bytes[C4M_K_OTHER] = 8.0 * cells * ((4 + (tracked ? 4 : 2)) + 2 * (2 + 2)) / 3.0;
    // Step 1: the step's E half, then Phi_J of Ez
    s = step_e_2d(p);
    if (s == C4M_OK) s = timed(p, C4M_K_OTHER, "source E", [&] { return group(C4M_EZ); });
    // Step 2: the step's H half, then Phi_J of Hx and Hy
    if (s == C4M_OK) s = step_h_2d(p);
    if (s == C4M_OK) s = timed(p, C4M_K_OTHER, "source Hx", [&] { return group(C4M_HX); });
    if (s == C4M_OK) s = timed(p, C4M_K_OTHER, "source Hy", [&] { return group(C4M_HY); });
    if (s != C4M_OK) return s;
    ++p->steps;
    return finite_check(p);
}

c4m_status c4m_get_info(c4m_problem* p, c4m_info* info)
{
    if (!p || !info) return fail(C4M_EINVAL, "null argument");
    memset(info, 0, sizeof(*info));
    info->steps = p->steps;
    info->tau_e = p->steps * p->cfg.cfl / p->N;
    info->tau_h = (p->steps + 0.5) * p->cfg.cfl / p->N;
    info->sweeps = p->cheb.sweeps;
    info->nonfinite = p->nonfinite;
    info->workspace_bytes = p->used;
    c4m_status s = flush_profile(p);
    if (s != C4M_OK) return s;
    if (p->pcg_state) {
        PcgState h{};
        hipError_t e = hipMemcpyAsync(&h, p->pcg_state, sizeof(h), hipMemcpyDeviceToHost, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return hip_fail(e, "PCG statistics");
        info->last_iters = h.last_iters;
        info->max_iters = h.max_iters;
        info->last_rel_residual = h.last_rel;
        info->noconv = h.noconv;
        info->sweeps = 0;
    }
    for (int k = 0; k < C4M_K_COUNT; ++k) {
        info->kernel_ms[k] = p->kernel_ms[k];
        info->kernel_launches[k] = p->kernel_launches[k];
        info->kernel_alg_bytes[k] = p->alg_bytes[k];
    }
    return C4M_OK;
}

c4m_status c4m_destroy(c4m_problem* p)
{
    if (!p) return fail(C4M_EINVAL, "null problem");
    if (p->owned_by_batch) return fail(C4M_ESTATE, "problem belongs to a batch");
    (void)flush_profile(p);
    drop_graphs(p);
    delete p;
    return C4M_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Hooks used by the batched form (c4m_batch.hip).
// ---------------------------------------------------------------------------
namespace c4m {

c4m_status set_error(c4m_status s, const char* msg) { return fail(s, msg); }

c4m_status problem_view(c4m_problem* p, ProblemView* v)
{
    for (int i = 0; i < 6; ++i) v->f[i] = p->f[i];
    for (int i = 0; i < 3; ++i) v->ge[i] = p->ge[i];
    for (int i = 0; i < 5; ++i) v->tmp[i] = p->tmp[i];
    v->yband = p->yband;
    v->used = p->used;
    v->N = p->N;
    v->P = p->P;
    for (int k = 0; k < 2; ++k) {
        v->line[k] = p->line[k];
        v->taps[k] = p->pade_host[k].taps;
    }
    v->coef = p->coef;
    v->cheb = p->cheb;
    return C4M_OK;
}

c4m_status problem_prepare(c4m_problem* p) { return ensure_ge(p); }

// The recorded 3D step of a member (null where the problem does not take that form).
const std::vector<Launch3>* problem_step3_plan(c4m_problem* p) { return plan3_form(p) ? &problem_plan3(p) : nullptr; }

c4m_status problem_create_owned(const c4m_config* cfg, void* ws, size_t bytes, hipStream_t st,
                                c4m_problem** out)
{
    c4m_status s = c4m_create(cfg, ws, bytes, (void*)st, out);
    if (s == C4M_OK) (*out)->owned_by_batch = true;
    return s;
}

void problem_add_steps(c4m_problem* p, int64_t n) { p->steps += n; }

// steps go to the stream directly (graph instantiation may allocate)
void problem_set_direct(c4m_problem* p) { p->direct = true; }

const c4m_config* problem_config(const c4m_problem* p) { return &p->cfg; }

void problem_destroy_owned(c4m_problem* p)
{
    (void)flush_profile(p);
    drop_graphs(p);
    delete p;
}
}  // namespace c4m
