// Batched kernel operators (K V on the matrix cores; many K_i v_i in one launch).
#pragma once

#include "kqr_internal.h"

namespace kqr {

// Launch shape of the K V kernel: nld = 0 streams 64-row tiles of K through
// LDS (row-contiguous loads); nld = 4 or 8 loads each strip's rows directly
// in the MFMA operand layout (16-byte loads per lane per step), with or
// without the next step's loads issued ahead; column segments.
constexpr int kKvMaxSegs = 8;
constexpr int kKvMaxCols = 16;  // right-hand sides of one K V launch
constexpr int kKvMaxExact = 4;  // exact (FP64) columns that ride along in one launch
constexpr int kKvBuckets = 8;
struct KvShape {
  int nld = 0;
  int prefetch = 1;
  int segs = 4;
};
KvShape default_kv_shape(int dtype, int64_t n);        // autotuned when set, else the default above
void set_kv_shape(int dtype, int64_t n, KvShape s);    // autotuner override (per dtype and size bucket)
bool kv_shape_supported(const KvShape& s);

// Doubles of scratch kapply_kv / kapply_kv_mixed need for n rows: the segment
// partials and, past them, the BF16 hi + lo parts of V (n x 32 halves); then
// the exact columns' segment partials and their FP64 copy (n x 4).
inline size_t kv_scratch_doubles(int64_t n) {
  return (size_t(kKvMaxSegs) + 1) * size_t(n) * 16 + (size_t(kKvMaxSegs) + 1) * size_t(n) * 4;
}

// U[:, j] = K V[:, j] for j < m <= 16.  V16: n_pad x 16 FP32 row-major (rows >= n
// and columns >= m zero); U: n x m FP64 (ld ldu); part: scratch of
// kv_scratch_doubles(n) doubles.
void kapply_kv(const KMat& km, int64_t n, const float* V16, int m, double* U, int64_t ldu, double* part,
               hipStream_t st, const KvShape* shape = nullptr);
struct SrcTable16 {
  const double* p[16];
};
struct DstTable16 {
  double* p[16];
};
// U[:, j] = K V16[:, j] (j < m, as kapply_kv, m may be 0) and, from the same
// pass over K, dst.p[j] = K src.p[j] for j < mx <= 4 with FP64 vectors,
// products and sums (the exact operator).  K: FP32, full layout.
void kapply_kv_mixed(const KMat& km, int64_t n, const float* V16, int m, double* U, int64_t ldu, SrcTable16 xsrc,
                     int mx, DstTable16 xdst, double* part, hipStream_t st);
// V16[i][j] = float(src.p[j][i]) for j < m, zero elsewhere (rows up to n_pad)
void kv_gather(SrcTable16 src, int m, int64_t n, int64_t n_pad, float* V16, hipStream_t st);
// V16[i][j] = float(V[i ldv + j]) for j < m, zero elsewhere
void kv_gather_strided(const double* V, int64_t ldv, int m, int64_t n, int64_t n_pad, float* V16, hipStream_t st);
// dst.p[j][i] = U16[i][j]
void kv_scatter(const double* U16, int m, int64_t n, DstTable16 dst, hipStream_t st);

// One problem of an uneven batch.
struct ProblemTask {
  const void* K;  // n x ld, FP32 or BF16
  int64_t ld;
  int64_t n;
  int dtype;
  const double* v;  // n (FP64; rounded to FP32 in the kernel, as every fast apply rounds v)
  double* u;       // n (FP64)
};
int problem_blocks(int64_t n);  // 32-row items of one problem

// u_t = K_t v_t for every task in one persistent launch whose workgroups take
// (problem, 32-row block) items from device counters (one per XCD, items
// interleaved over them).  The task table goes
// to the device through a ring of pinned staging copies, so a launch does not
// wait for the host.  Launches must be ordered on one stream.
constexpr int kQueueCounters = 8;  // item counters of the problem queue (one per XCD)

class ProblemQueue {
 public:
  explicit ProblemQueue(size_t max_tasks);
  ~ProblemQueue();
  ProblemQueue(const ProblemQueue&) = delete;
  ProblemQueue& operator=(const ProblemQueue&) = delete;
  void launch(const std::vector<ProblemTask>& tasks, hipStream_t st);

 private:
  static constexpr int kRing = 8;
  static constexpr int kQueueWgs = 2048;  // resident workgroups: 256 CUs x 8
  size_t cap_, slot_bytes_;
  DevBuf table_;
  HostPinned stage_;
  DevBuf ctr_;
  hipEvent_t copied_[kRing] = {};
  bool used_[kRing] = {};
  uint64_t base_[kQueueCounters] = {};
  int next_ = 0;
};

}  // namespace kqr
