// Arguments of the cooperative FP64 Hermitian eigensolver (eigen.hip), shared
// by the clutter filter's driver (svd.hip).
#pragma once

#include "common.h"

namespace ulm {

constexpr int kCoopMaxW = 32;      // work-groups per plane (one barrier flag each)
constexpr int kPlaceWord = kBarStride - 1;  // per-plane word: bit x set by a work-group on XCC x

struct EigArgs {
    const double2 *C;   // [planes][F][F] covariance (full Hermitian)
    double2 *H;         // [planes][F][F] row k: Householder vector v_k (entries k+1..F-1)
    double2 *tau;       // [planes][F]
    double *d, *e;      // [planes][F]
    double *lam;        // [planes][F] eigenvalues, descending
    double *lam_out;    // optional copy of lam
    double2 *V;         // [planes][F][c] clutter eigenvectors
    double *tscr;       // [planes][c][6][F]
    double2 *xscr;      // [planes][c][F]
    double2 *vbuf;      // [planes][2][F] published columns (double-buffered by step parity)
    double2 *pbuf;      // [planes][2][F] published p = tau A v
    int *bar;           // [planes][kBarStride] barrier flags and the XCC mask, zero at launch
    int *flag;          // [planes] non-finite input
    int *status;
    int F, c, W;
    int agent_scope;    // nonzero: the fenced mode even when a plane is on one XCD
    int planes;         // solve planes [plane0, planes)
    int plane0;
};

int eigen_coop_width(int F);
size_t eigen_coop_lds(int F, int c);
hipError_t launch_eigen_coop(const EigArgs &args, hipStream_t st);

}  // namespace ulm
