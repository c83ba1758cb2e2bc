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
// unknown box (inclusive), the pitch and the constants of M.
struct ChebGeom {
    int n[2], half[2], lo[2], hi[2], P;
    double alpha, beta;
};

// Field update of the last Chebyshev application (field == nullptr: none).
struct SrcUpdate {
    double* field;
    double* ge;                 // G_E with the carried Laplacian, else nullptr
    const double* jz;           // F_J of the G_E update
    const double* jz_tt;
    double r, z, ht2, ge_gain, ge_src;
};

// Arguments of one component's correction launch (comp 2: Ez, 0: Hx, 1: Hy).
struct SrcTile {
    SourceTM s;
    const double* cols;         // Ez: column 0 of A^{-1}, half->node; Hx, Hy: node->half
    SrcCoef c;
    ChebGeom g;
    SrcUpdate u;
    int comp, N, K;             // K: applications of M (the problem's schedule)
    double w[MAX_SWEEPS + 1];   // step sizes of the first-order form (the launcher fills them)
};

hipError_t launch_src_group(hipStream_t st, const SrcTile& a);

}  // namespace c4m
