// Batched PCG steps (pstep.h): staging of the descriptor tables and the
// sequence of the five launches.
#include "pstep.h"

#include <cstring>

namespace kqr {

namespace {
size_t align256(size_t b) { return (b + 255) / 256 * 256; }
size_t step_table_bytes(size_t cap) {
  return align256(cap * sizeof(PcgStepDesc)) + 3 * align256((cap + 1) * sizeof(int));
}
}  // namespace

PcgStepBatch::PcgStepBatch(size_t max_fits)
    : cap_(std::max<size_t>(max_fits, 1)), slot_bytes_(step_table_bytes(cap_)), table_(kRing * slot_bytes_),
      stage_(kRing * slot_bytes_) {
  for (auto& e : copied_) KQR_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

PcgStepBatch::~PcgStepBatch() {
  for (auto& e : copied_) (void)hipEventDestroy(e);
}

void PcgStepBatch::launch(const std::vector<PcgStepDesc>& steps, hipStream_t st) {
  if (steps.empty()) return;
  if (steps.size() > cap_) fail(KQR_EHIP, "internal: %zu PCG steps for a table of %zu", steps.size(), cap_);
  const int k = next_;
  next_ = (next_ + 1) % kRing;
  // the staging copy of this ring slot was last read by the copy recorded kRing launches ago
  if (used_[k]) KQR_CHECK_HIP(hipEventSynchronize(copied_[k]));
  char* stage = static_cast<char*>(stage_.ptr) + size_t(k) * slot_bytes_;
  char* table = static_cast<char*>(table_.ptr) + size_t(k) * slot_bytes_;
  const int nf = int(steps.size());
  const size_t desc_bytes = align256(cap_ * sizeof(PcgStepDesc)), first_bytes = align256((cap_ + 1) * sizeof(int));
  // fits whose vectors fit one workgroup first (n1 of them), then the longer ones
  PcgStepDesc* sd = reinterpret_cast<PcgStepDesc*>(stage);
  int n1 = 0;
  for (const PcgStepDesc& e : steps)
    if (e.nred == 1) sd[n1++] = e;
  int m = n1;
  for (const PcgStepDesc& e : steps)
    if (e.nred > 1) sd[m++] = e;
  const int n2 = nf - n1;
  int* gt_first = reinterpret_cast<int*>(stage + desc_bytes);
  int* fs_first = reinterpret_cast<int*>(stage + desc_bytes + first_bytes);
  int* red_first = reinterpret_cast<int*>(stage + desc_bytes + 2 * first_bytes);
  int gt_total = 0, fs_total = 0, red_total = 0;
  for (int f = 0; f < nf; ++f) {
    gt_first[f] = gt_total;
    fs_first[f] = fs_total;
    gt_total += pcg_step_gt_blocks(sd[f]);
    fs_total += pcg_step_fs_blocks(sd[f]);
  }
  gt_first[nf] = gt_total;
  fs_first[nf] = fs_total;
  for (int f = 0; f < n2; ++f) {
    red_first[f] = red_total;
    red_total += sd[n1 + f].nred;
  }
  red_first[n2] = red_total;
  KQR_CHECK_HIP(hipMemcpyAsync(table, stage, slot_bytes_, hipMemcpyHostToDevice, st));
  KQR_CHECK_HIP(hipEventRecord(copied_[k], st));
  used_[k] = true;
  const auto* d = reinterpret_cast<const PcgStepDesc*>(table);
  const auto* d2 = d + n1;
  const int* red = reinterpret_cast<const int*>(table + desc_bytes + 2 * first_bytes);
  // q, x, r, K x and r . r
  launch_pcg_qxr_steps(d, n1, st);
  launch_pcg_q_steps(d2, red, n2, red_total, st);
  launch_finalize_steps(d2, n2, 0, st);
  launch_pcg_xr_steps(d2, red, n2, red_total, st);
  launch_finalize_steps(d2, n2, 1, st);
  // zz = P^{-1} r: F^T g, the core solve, F s for every fit
  launch_wood_gt_steps(d, reinterpret_cast<const int*>(table + desc_bytes), nf, gt_total, st);
  launch_core_solve_steps(d, nf, st);
  launch_wood_fs_steps(d, reinterpret_cast<const int*>(table + desc_bytes + first_bytes), nf, fs_total, st);
  // the output, r . zz, the direction update and sum p
  launch_wood_out_p_steps(d, n1, st);
  launch_wood_out_steps(d2, red, n2, red_total, st);
  launch_finalize_steps(d2, n2, 2, st);
  launch_pcg_p_steps(d2, red, n2, red_total, st);
  launch_finalize_steps(d2, n2, 3, st);
}

}  // namespace kqr
