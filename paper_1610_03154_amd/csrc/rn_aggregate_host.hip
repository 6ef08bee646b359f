// rn_aggregate_host.hip -- standard greedy aggregation with root nodes
// (Sec. 3.3) on the host.  The GPU path takes the aggregation as input; this
// helper lets a caller produce it from the strength graph of rn_strength.
//
// Sweep 1 visits nodes in index order; a node becomes a root when it and all
// its strong neighbours are free, and its aggregate is the node plus those
// neighbours.  Sweep 2 gives each free node the aggregate of its first
// (lowest-index) strong neighbour that sweep 1 placed.  Sweep 3 turns every
// node still free into a root of a new aggregate with its free neighbours.
#include <cstdint>
#include <vector>

#include "rnamg.h"

extern "C" rn_status rn_aggregate_host(int32_t nn, const int32_t *Sp, const int32_t *Sj, int32_t *agg,
                                       int32_t *roots, int32_t *n_agg) {
  if (nn < 0 || !n_agg || (nn > 0 && (!Sp || !Sj || !agg || !roots))) return RN_EINVAL;
  const int64_t nz = nn > 0 ? Sp[nn] : 0;
  if (nn > 0 && Sp[0] != 0) return RN_EINVAL;
  for (int32_t i = 0; i < nn; ++i)
    if (Sp[i + 1] < Sp[i] || Sp[i + 1] > nz) return RN_EINVAL;
  for (int64_t p = 0; p < nz; ++p)
    if (Sj[p] < 0 || Sj[p] >= nn) return RN_EINVAL;
  int32_t na = 0;
  for (int32_t i = 0; i < nn; ++i) agg[i] = -1;
  for (int32_t i = 0; i < nn; ++i) {
    if (agg[i] != -1) continue;
    bool all_free = true;
    for (int32_t p = Sp[i]; p < Sp[i + 1] && all_free; ++p) all_free = (Sj[p] == i) || (agg[Sj[p]] == -1);
    if (!all_free) continue;
    roots[na] = i;
    agg[i] = na;
    for (int32_t p = Sp[i]; p < Sp[i + 1]; ++p) agg[Sj[p]] = na;
    ++na;
  }
  const std::vector<int32_t> placed(agg, agg + nn);
  for (int32_t i = 0; i < nn; ++i) {
    if (agg[i] != -1) continue;
    for (int32_t p = Sp[i]; p < Sp[i + 1]; ++p) {
      const int32_t j = Sj[p];
      if (j != i && placed[j] != -1) {
        agg[i] = placed[j];
        break;
      }
    }
  }
  for (int32_t i = 0; i < nn; ++i) {
    if (agg[i] != -1) continue;
    roots[na] = i;
    agg[i] = na;
    for (int32_t p = Sp[i]; p < Sp[i + 1]; ++p)
      if (agg[Sj[p]] == -1) agg[Sj[p]] = na;
    ++na;
  }
  *n_agg = na;
  return RN_OK;
}
