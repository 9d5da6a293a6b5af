// One PCG iteration's work after its K-apply, batched over the fits of a
// rendezvous round.
//
// A PCG iteration (Algorithm 3's linear solves, preconditioned with the
// Woodbury form of Lemma 1) is, once K p is known:
//   q = K p + c 1 (1^T p) + L p,  a = rz / (p . q),
//   x += a p,  r -= a q,  K x += a K p,  rr = r . r          (pcg_qxr)
//   zz = P^{-1} r  (g = r / L, t = [U 1]^T g, s = C^{-1} t,
//                   zz = g - (U s_{1..r} + s_{r+1}) / L)     (Woodbury apply)
//   rz' = r . zz,  p = zz + (rz' / rz) p,  sum(p)           (direction update)
// For a fit whose core is small (r + 1 <= kFusedCore) every step above is a
// launch or two of single-fit kernels: one launch each when the vectors fit
// one workgroup (n <= kOneBlockN), else a pass over several workgroups whose
// partial sums a finishing launch adds.  A batch runs the same device bodies
// once per fit from a table of these descriptors -- five launches when every
// fit's vectors fit one workgroup, up to thirteen when some are longer -- so
// the sums and their order, and the results, are those of the single-fit
// launches.  The preconditioner runs before the fit has read rr: when rr says
// the solve has converged (or p . q <= 0), the fit drops zz and p.
#pragma once

#include <vector>

#include "kqr_internal.h"

namespace kqr {

// Woodbury cores up to this order are solved in one workgroup (core_solve).
constexpr int kFusedCore = 128;

struct PcgStepDesc {
  int64_t n = 0;
  // pcg_qxr
  const double* Kp = nullptr;
  const double* L = nullptr;  // the system's diagonal
  double c = 0.0;
  double* sc = nullptr;  // the solve's scalar slots
  int sump = 0, rz = 0, pq = 0, rr = 0, rz_new = 0;
  double* q = nullptr;
  double* x = nullptr;
  double* r = nullptr;
  double* Kx = nullptr;  // may be null
  double* p = nullptr;
  float* p32 = nullptr;  // may be null
  // Woodbury apply (zz = P^{-1} r)
  const double* Lw = nullptr;  // the preconditioner's diagonal
  const float* F = nullptr;  // n x rank, leading dimension ldf (null when rank = 0)
  int64_t ldf = 0;
  int rank = 0;
  int R1 = 1;  // rank + 1 <= kFusedCore
  int nblk = 1;  // workgroups of the F^T g pass
  int64_t chunk = 0;  // rows per workgroup of that pass
  double* g = nullptr;
  double* part = nullptr;  // nblk x R1 partial sums of F^T g
  const double* W = nullptr;  // core inverse factor and its transpose
  const double* WT = nullptr;
  int64_t ldc = 0;
  double* s = nullptr;
  double* Fs = nullptr;
  double* zz = nullptr;
  // vectors longer than one workgroup: the blocks of each pass (red_shape) and
  // the fit's partial sums (nred = 1: the one-workgroup kernels, no partials)
  int nred = 1;
  double* partials = nullptr;
  // optional pinned host triple: (p . q, r . r) written at the end of the
  // step, then (after a system-scope fence) 1 into the third entry, which the
  // fit's host thread has set to 0 before handing the step in
  double* status = nullptr;
};

// Device tables of the batched launches: the descriptors and, per fit, the
// first workgroup of its F^T g pass and of its F s pass (prefix sums, with
// the totals at the end), in a ring of staging copies (no host wait).
class PcgStepBatch {
 public:
  explicit PcgStepBatch(size_t max_fits);
  ~PcgStepBatch();
  PcgStepBatch(const PcgStepBatch&) = delete;
  PcgStepBatch& operator=(const PcgStepBatch&) = delete;
  void launch(const std::vector<PcgStepDesc>& steps, hipStream_t st);

 private:
  static constexpr int kRing = 8;
  size_t cap_, slot_bytes_;
  DevBuf table_;
  HostPinned stage_;
  hipEvent_t copied_[kRing] = {};
  bool used_[kRing] = {};
  int next_ = 0;
};

// The batched launches (each in the translation unit of its single-fit
// kernel).  d: nf device descriptors; gt_first / fs_first: nf + 1 prefix sums
// of the per-fit workgroup counts.  The first five serve fits of one workgroup
// (the Woodbury passes serve every fit).
void launch_pcg_qxr_steps(const PcgStepDesc* d, int nf, hipStream_t st);
void launch_wood_gt_steps(const PcgStepDesc* d, const int* gt_first, int nf, int total, hipStream_t st);
void launch_core_solve_steps(const PcgStepDesc* d, int nf, hipStream_t st);
void launch_wood_fs_steps(const PcgStepDesc* d, const int* fs_first, int nf, int total, hipStream_t st);
void launch_wood_out_p_steps(const PcgStepDesc* d, int nf, hipStream_t st);
// the passes of fits longer than one workgroup (red_first: prefix of their nred)
void launch_pcg_q_steps(const PcgStepDesc* d, const int* red_first, int nf, int total, hipStream_t st);
void launch_pcg_xr_steps(const PcgStepDesc* d, const int* red_first, int nf, int total, hipStream_t st);
void launch_wood_out_steps(const PcgStepDesc* d, const int* red_first, int nf, int total, hipStream_t st);
void launch_pcg_p_steps(const PcgStepDesc* d, const int* red_first, int nf, int total, hipStream_t st);
// the finishing sums, one workgroup per fit: which = 0 p.q, 1 r.r, 2 r.zz, 3 sum p (+ status)
void launch_finalize_steps(const PcgStepDesc* d, int nf, int which, hipStream_t st);

// Workgroup counts of the two multi-workgroup passes for one fit.
int pcg_step_gt_blocks(const PcgStepDesc& d);
int pcg_step_fs_blocks(const PcgStepDesc& d);

// The fit whose workgroups [first[f], first[f + 1]) hold block b (first has nf + 1 entries).
__device__ __forceinline__ int step_of_block(const int* __restrict__ first, int nf, int b) {
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace kqr
