// Preparation products of a block (Sec. IV A): for the k_ins candidates,
//   YT = (N Z)^T   (G of old rows, candidate columns),
//   Rt = X N       (candidate rows of the augmented N, the paper's R~),
//   Gnn = X Y + G0nn (G of candidate rows and columns).
// Each of YT and Rt reads N once; both run as skinny MFMA products (k_skinny.hip).
#include "ctaux_device.h"

namespace ctaux {

void launch_skinny(const Batch &b, hipStream_t s, int kind);

void launch_prep(const Batch &b, hipStream_t s) {
  launch_skinny(b, s, 0);   // YT = ZT N^T, Rt = X N
  launch_skinny(b, s, 1);   // Gnn = X YT^T + G0nn
}

}  // namespace ctaux
