// c4m_source.h -- device-side types of the sourced 2D (TM) step
// (c4m_source.hip) and its launchers.
#pragma once

#include "c4m_internal.h"

namespace c4m {

using SourceTM = c4m_source_tm;

struct SrcCoef {
    double h, ht2, h2_24;   // h, h_t^2 / 24, h^2 / 24
    double alpha, beta, z;
};

// One component grid of the correction solve: extents, half flags, the
// unknown box (inclusive) and the M / Chebyshev constants.
struct ChebGeom {
    int n[2], half[2], lo[2], hi[2], P;
    double alpha, beta, inv_theta;
};

// Field update of the last Chebyshev application (field == nullptr: none).
struct SrcUpdate {
    double* field;
    double* ge;                 // G_E with the carried Laplacian, else nullptr
    const double* jz;           // F_J of the G_E update
    const double* jz_tt;
    double r, z, ht2, ge_gain, ge_src;
};

hipError_t launch_src_rhs_e(hipStream_t st, double* b, const SourceTM& s, const double* wc, int N, int P,
                            const SrcCoef& c);
hipError_t launch_src_rhs_h(hipStream_t st, double* b, const SourceTM& s, const double* vc, int comp, int N,
                            int P, const SrcCoef& c);
hipError_t launch_src_solve(hipStream_t st, const double* b, double* xa, double* xb, const ChebGeom& g,
                            const ChebSchedule& cs, const SrcUpdate& u);

}  // namespace c4m
