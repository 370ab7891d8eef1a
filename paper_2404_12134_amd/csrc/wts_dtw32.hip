// wts_dtw32.hip -- the float32-decision instances of the DTW sweep
// (wts_sweep.h with a float32 compute type): the recurrence, its minima and
// the argmin codes in float32 on float32 cycles and the barycenter rounded to
// float32.  A translation unit of its own so the two sets compile in parallel.
#include "wts_sweep.h"

namespace wts {

hipError_t launch_fwd32(int d, int rho, int mode, bool euc, bool x_is_cycle, int ydtype,
                        const FwdArgs& a, int grid, hipStream_t st) {
  return launch_fwd_impl<float>(d, rho, mode, euc, x_is_cycle, ydtype, a, grid, st);
}

}  // namespace wts
