// Batched PCG steps (pstep.h): staging of the descriptor tables and the
// sequence of the five launches.
#include "pstep.h"

#include <cstring>

namespace kqr {

namespace {
size_t align256(size_t b) { return (b + 255) / 256 * 256; }
size_t step_table_bytes(size_t cap) {
  return align256(cap * sizeof(PcgStepDesc)) + 2 * align256((cap + 1) * sizeof(int));
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
  memcpy(stage, steps.data(), steps.size() * sizeof(PcgStepDesc));
  int* gt_first = reinterpret_cast<int*>(stage + desc_bytes);
  int* fs_first = reinterpret_cast<int*>(stage + desc_bytes + first_bytes);
  int gt_total = 0, fs_total = 0;
  for (int f = 0; f < nf; ++f) {
    gt_first[f] = gt_total;
    fs_first[f] = fs_total;
    gt_total += pcg_step_gt_blocks(steps[size_t(f)]);
    fs_total += pcg_step_fs_blocks(steps[size_t(f)]);
  }
  gt_first[nf] = gt_total;
  fs_first[nf] = fs_total;
  KQR_CHECK_HIP(hipMemcpyAsync(table, stage, slot_bytes_, hipMemcpyHostToDevice, st));
  KQR_CHECK_HIP(hipEventRecord(copied_[k], st));
  used_[k] = true;
  const auto* d = reinterpret_cast<const PcgStepDesc*>(table);
  launch_pcg_qxr_steps(d, nf, st);
  launch_wood_gt_steps(d, reinterpret_cast<const int*>(table + desc_bytes), nf, gt_total, st);
  launch_core_solve_steps(d, nf, st);
  launch_wood_fs_steps(d, reinterpret_cast<const int*>(table + desc_bytes + first_bytes), nf, fs_total, st);
  launch_wood_out_p_steps(d, nf, st);
}

}  // namespace kqr
