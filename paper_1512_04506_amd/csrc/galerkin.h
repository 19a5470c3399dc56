// Galerkin assembly of the block-crossing couplings of D_c straight from the
// aggregate basis (no intermediate D P field).
#pragma once
#include "ddamg_internal.h"

namespace ddamg {

// Largest number of test vectors the fused crossing-piece kernel handles
// (one 32-wide matrix-core tile per chirality).
constexpr int GALERKIN_CROSS_MAX_NTV = 32;

// Writes the forward slots 1 + 2 mu (mu = 0..3) of every coarse site of
// Dc [Nb][9][col][row] (precision T, FP32 or FP64) from the stored basis bv
// and the links in T.  Requires g.ntv <= GALERKIN_CROSS_MAX_NTV; other slots
// are left alone.
template <typename T, typename S>
void launch_galerkin_cross(cx<T>* Dc, const BasisView<S>& bv, const GaugeView<T>& gv, const Geom& g, hipStream_t st);

}  // namespace ddamg
