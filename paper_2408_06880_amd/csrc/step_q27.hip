// AA step kernels, D3Q27 (SRT, TRT, cumulant; all storages).
#include "internal.hpp"
#include "step_impl.hpp"

namespace lbm {

hipError_t launch_aa_q27(int coll, int storage, int mode, int idx, const StepArgs& a,
                         int block, uint32_t lds, bool links, hipStream_t st) {
  switch (coll) {
    case COLL_NONE: return launch_aa_c<27, COLL_NONE>(storage, mode, idx, a, block, lds, links, st);
    case COLL_SRT: return launch_aa_c<27, COLL_SRT>(storage, mode, idx, a, block, lds, links, st);
    case COLL_TRT: return launch_aa_c<27, COLL_TRT>(storage, mode, idx, a, block, lds, links, st);
    case COLL_CUMULANT: return launch_aa_c<27, COLL_CUMULANT>(storage, mode, idx, a, block, lds, links, st);
    case COLL_CM: return launch_aa_c<27, COLL_CM>(storage, mode, idx, a, block, lds, links, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
