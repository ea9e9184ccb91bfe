// amm_gen.h -- interface to the generated straight-line integrand kernels.
#pragma once
#include "amm_kernels.h"

namespace amm {

enum GenKind { GEN_RUN = 0, GEN_EVAL = 1 };

// One launcher per (loop order, graph): GEN_RUN launches the FP64 pass of a
// chunk batch; GEN_EVAL evaluates given points in FP64 with bounds.  The
// double-double recompute always uses the table interpreter.
using GenLaunchFn = void (*)(int kind, const DensityDev *D, const RunArgs *A, int grid, const double *z, uint64_t n,
                             double *I, double *absI, double *bound, hipStream_t s, double *part, uint32_t *flag,
                             int32_t *nflag);

// Launcher of graph g of the given loop order, or nullptr when no generated
// code was built for it (the table interpreter is used then).
GenLaunchFn gen_launch(int loops, int g);

}  // namespace amm
