// c4m_internal.h -- shared between the host runtime and the gfx950 kernels.
//
// Device layout: every field of a problem lives in one padded array shape,
// (nz, ny, P) with row pitch P = round_up(N + 1, 16) doubles and ny = N + 1
// (nz = N + 1 in 3D, 1 in 2D), so all components share the strides
// sy = P and sz = (N + 1) P and differ only in their valid extents.
#pragma once

#include <hip/hip_runtime.h>
#include <vector>
#include <stdint.h>

#include "c4m.h"

namespace c4m {

// Truncated inverse of the Pade matrix A (Appendix A.1, eq:lhs).  The
// interior rows of A^{-1} decay like |rho|^k with rho = -11 + sqrt(120)
// (|rho| ~ 0.0455), so entries beyond |k| = PADE_R (< 5e-18 relative) are
// dropped.  Folding the two-point difference D into the rows gives
// 2 PADE_R + 2 taps on the undifferenced line values.
constexpr int PADE_R = 12;
constexpr int PADE_TAPS = 2 * PADE_R + 2;
constexpr int PADE_B = 2 * PADE_R;   // explicit rows at each end of a line
// Rows of the derivative of the conditioned source alpha f + (second
// difference of f along the line) / 12, folded into taps on the raw values
// f[m-R-1 .. m+R+2] (the end rules of the conditioning included).
constexpr int COND_TAPS = PADE_TAPS + 2;
// Interior rows are antisymmetric about m + 1/2: tap pairs on
// f[m-j] - f[m+1+j], j = 0 .. COND_TAPS/2 - 1 (conditioned) and
// j = 0 .. PADE_TAPS/2 - 1 (raw), stored after the conditioned rows.
constexpr int PAIR_TAPS = COND_TAPS / 2 + PADE_TAPS / 2;
// Rows per end of the band table of the 2D strip form (room for every row
// of a short line).
constexpr int YB_ROWS = 2 * PADE_B;

struct PadeTaps {
    double c[PADE_TAPS];             // interior (Toeplitz) row, tap u at c[u + PADE_R]
};

// Device view of one line kind (a given n_in and node/half orientation).
// Rows m < b and m >= n_out - b use rows[] (b rows at each end, stored left
// block then right block, then the interior row); if `all` is set every
// row is explicit (short lines) and rows[m] is row m.  crows has the same
// row order with COND_TAPS taps per row; pairs holds the interior pair taps
// (conditioned first).
struct PadeLine {
    const double* rows;              // [n_rows][PADE_TAPS]
    int n_in, n_out, b, all;
    const double* crows;             // [n_rows][COND_TAPS]
    const double* pairs;             // [PAIR_TAPS]
};

// Spectral bounds of M = alpha I - beta L9: [alpha, alpha + 16/3 beta]
// (symbol S in [0, 16/3], Appendix A.2); Chebyshev schedule on them.
constexpr int MAX_SWEEPS = 8;
// Default number of applications: the fewest whose Chebyshev contraction
// 1 / T_{K+1}(sigma) is below CHEB_TOL, about two units in the last place
// of FP64 (below the CG tolerance of the paper's solver, so the solve is
// exact to rounding): five at r = 0.5 in 2D, four at r = 0.4 in 3D.
constexpr double CHEB_TOL = 4e-16;
struct ChebSchedule {
    double inv_theta;                // 1 / theta, theta = (lmax + lmin) / 2
    double c1[MAX_SWEEPS];           // d <- c1 d + c2 r after apply k
    double c2[MAX_SWEEPS];
    float c1f[MAX_SWEEPS];
    float c2f[MAX_SWEEPS];
    float inv_thetaf;
    int sweeps;
};

// Unknown range of one component grid along x, y, z and the boundary type:
// Dirichlet (node axis, walls excluded, value 0 beyond) or Neumann (half
// axis, even ghost).
struct UGrid {
    int lo[3], hi[3];
    int neumann[3];
};

// Extent and half-point flags of one component on the common padded layout.
struct Box {
    int n[3];
    int half[3];
    int active[3];
};

struct Coef {
    double alpha, beta, cfl, z;
    double ge_gain;                  // 1 + 4/r^2 : G_E += ge_gain * dE - ...
    double ge_curl;                  // (2/r) Z   : ... - ge_curl * curl^A H
};

// 3D: one Pade line-derivative term accumulated into a target right-hand side.
struct Term3 {
    const double* src;
    double* out;
    Box sb;            // source component extents and half flags
    UGrid tg;          // target unknown ranges (outputs along the line start at tg.lo[axis])
    int P;
    size_t plane;
    double scale;
    int accumulate;
};

// 3D: arrays of one Chebyshev solve (r holds b on entry).
struct Cheb3 {
    double* r;
    double* x;
    double* d0;
    double* d1;
    UGrid g;
    int P;
    size_t plane;
};

// 3D Chebyshev pass (c4m_kernels_3d.hip).
enum { C3_STORE = 0, C3_FIELD = 1, C3_RESID = 2 };
// TX: storage of the iterates, TB: storage of b.
template <class TX, class TB>
struct Cheb3T {
    const TB* b;
    const TX* xk;           // x_k (unused in the first pass: x_1 = b / theta)
    const TX* xkm1;         // x_{k-1} (first pass: x_0 = 0; second pass: x_1 = b / theta, formed here)
    TX* xout;               // C3_STORE: x_{k+1}
    const TX* xadd;         // C3_FIELD: an earlier round's solution added to Phi (or null)
    float* rout;            // C3_RESID: b - M x_k, rounded to FP32
    double* field;          // C3_FIELD: field += cfl Phi
    double* ge;             // C3_FIELD, carried Laplacian: G_E update (or null)
    const double* cur;      // raw curl for the G_E update
    UGrid g;
    int P;
    size_t plane;
    double inv_theta, c1, c2;
    Coef cf;
};

// One launch of the 3D step of one problem (FP64 Chebyshev form), recorded
// once per problem: the single-problem step launches the records in order,
// the batched step launches each record over all members at once.
enum { L3_COND = 0, L3_TERM = 1, L3_MARCH = 2, L3_CHEB = 3 };
struct Launch3 {
    int kind;               // L3_*
    int axis, mode;         // term / march: line axis; cond: source mode
    int line;               // Pade line (taps) of a term
    int first, out;         // cheb: first pass, output kind
    int cls, group;         // kernel class and component (profiling groups)
    Term3 t;
    PadeLine L;
    int seg;                // march: outputs per wave
    Cheb3T<double, double> c;
    unsigned gx, gy, gz;    // this problem's grid of the launch
};
// What the planner needs of a problem.
struct Plan3In {
    double* f[6];
    double* ge[3];
    double* tmp[8];
    Box box[6];
    UGrid ug[6];
    int P;
    size_t plane;
    Coef coef;
    ChebSchedule cheb;
    PadeLine line[2];
    bool tracked;
};
void plan_step3(const Plan3In& in, std::vector<Launch3>& out);
hipError_t launch3_single(hipStream_t st, const Launch3& r, const PadeTaps* taps);
size_t launch3_arg_bytes(const Launch3& r);
void launch3_pack(const Launch3& r, int first_block, void* dst);
hipError_t launch3_batched(hipStream_t st, const Launch3& proto, const void* dev_args, int count,
                           unsigned total_blocks, const PadeTaps* taps);

// Device tables of the transform solve for one N (c4m_transform.hip):
// orthonormal DST-I (N-1 x N-1), DCT-II (N x N) and its transpose, sigma.
struct TransformTables {
    const double* S;
    const double* C;
    const double* Ct;
    const double* sig_d;
    const double* sig_n;
};
size_t transform_table_doubles(int N);
void build_transform_tables(int N, double* host, TransformTables* t, double* dev);
hipError_t launch_transform_solve(hipStream_t st, int dim, const TransformTables& t, const UGrid& g, int P,
                                  size_t plane, const double* b, double* w1, double* w2, double* field, double* ge,
                                  const double* cur, const Coef& cf);

// PCG solve state on the device (one per problem).
struct PcgState {
    int arrived;          // workgroups that published their partials (reset by the last)
    int done;             // residual target met: later kernels of the solve return at once
    int iters;            // iterations of the current solve
    int last_iters, max_iters, noconv;
    double rz, bb, rr;    // <r, z>, <b, b>, <r, r>
    double alpha, beta;   // step lengths of the current iteration
    double last_rel;      // sqrt(rr / bb) at the end of the last solve
};

// Arrays of one PCG solve on one component grid (b in r on entry).
struct PcgArgs {
    double* x;
    double* r;
    double* p[2];         // search directions (alternate per iteration)
    double* q;            // M p
    double* dinv;         // 1 / diag(M)
    double* z;            // preconditioned residual r / diag(M)
    double* part;         // [3][nparts] per-workgroup partial sums
    PcgState* st;
    UGrid g;
    int P;
    size_t plane;
    int nparts;
    double alpha, beta;   // M = alpha I - beta L9
    double rtol2;         // squared relative residual target
};

// One PCG solve (c4m_pcg.hip): M x = b with b in a.r (overwritten), at most
// max_iter iterations, then field += cfl x (and the G_E update when ge is
// given, with cur the raw curl).  dim 2 uses the 9-point L9, dim 3 the
// 19-point one.
hipError_t launch_pcg(hipStream_t st, int dim, PcgArgs a, int max_iter, double* field, double* ge,
                      const double* cur, const Coef& cf);
size_t pcg_partials(const UGrid& g);

// Internal view of a problem for the batched form (c4m_host.hip fills it).
struct ProblemView {
    double* f[6];
    double* ge[3];
    double* tmp[5];
    double* yband;        // 2D band table of the strip form
    size_t used;          // workspace bytes in use (one buffer resource must span them)
    int N, P;
    PadeLine line[2];
    PadeTaps taps[2];
    Coef coef;
    ChebSchedule cheb;
};

}  // namespace c4m
