// The Toeplitz normal operator's kernels for one padded transform length
// N = 2 * MRX_N2 * MRX_N3, built with
//   -DMRX_N2=.. -DMRX_N3=.. -DMRX_T=.. -DMRX_TWR=.. -DMRX_TWC=.. -DMRX_NAME=".."
// (T threads a transform, TWR rows a workgroup in the row passes, TWC
// columns a workgroup in the column pass).  Registers them when the library
// is loaded.
#include "toeplitz.h"

namespace mrx {
namespace {
RegistrarToep<Sched<2, MRX_N2, MRX_N3, MRX_T>, MRX_TWR, MRX_TWC> registrar_toep_(MRX_NAME);
}  // namespace
}  // namespace mrx
