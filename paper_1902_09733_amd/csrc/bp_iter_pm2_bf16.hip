// The fused pair of half-sweeps (bp_iter_pm2_impl.h) with BF16 message storage.
#include "bp_iter_pm2_impl.h"

namespace bpk {

template bp_status pm2_single<StoreBF16>(const PairArgs &, size_t, int, int, bool, hipStream_t);
template bp_status pm2_batch<StoreBF16>(const PairEntry *, int, int, size_t, int, int, bool, bool, int, hipStream_t);

}  // namespace bpk
