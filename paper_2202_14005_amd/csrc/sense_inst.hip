// One transform schedule for one length, selected by the build with
//   -DMRX_N1=.. -DMRX_N2=.. -DMRX_N3=.. -DMRX_T=.. -DMRX_WTC=.. -DMRX_WTR=.. -DMRX_G=.. -DMRX_KS=0|1 -DMRX_NAME=".."
// and -DMRX_WL=1 for the wave-local normal operator (k_normal_wl), =2 for it
// with the padded LDS layout; -DMRX_KSPL=k splits a column tile's coils over
// k workgroups in CG steps; -DMRX_SOFT=1 also registers the length's
// soft-SENSE kernels on this decomposition (-DMRX_SOFT_WTN=.. the soft
// normal operator's tile width, default MRX_WTC).
// It registers its column and row kernels with the schedule registry when
// the library is loaded.
#include "sense_soft.h"

namespace mrx {
namespace {
#if defined(MRX_WL) && MRX_WL
RegistrarWL<Sched<MRX_N1, MRX_N2, MRX_N3, MRX_T>, MRX_WTC, MRX_WTR, MRX_G, (MRX_WL == 2)> registrar_(MRX_NAME);
#else
#ifndef MRX_KSPL
#define MRX_KSPL 1
#endif
Registrar<Sched<MRX_N1, MRX_N2, MRX_N3, MRX_T>, MRX_WTC, MRX_WTR, MRX_G, (MRX_KS != 0), MRX_KSPL> registrar_(MRX_NAME);
#endif
#if defined(MRX_SOFT) && MRX_SOFT
// the length's soft-SENSE kernels, on this schedule's decomposition and
// column tile (one schedule per length carries them)
#ifndef MRX_SOFT_WTN
#define MRX_SOFT_WTN MRX_WTC
#endif
RegistrarSoft<Sched<MRX_N1, MRX_N2, MRX_N3, MRX_T>, MRX_SOFT_WTN, MRX_WTC> registrar_soft_(MRX_NAME);
#endif
}  // namespace
}  // namespace mrx
