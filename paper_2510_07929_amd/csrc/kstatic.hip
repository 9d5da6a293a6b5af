// K-apply that allocates nothing: the materialised single-vector K v of
// kqr_kernel_apply with its scratch (the FP32 copy of v, an aligned FP64 copy
// when v is strided, the column-segment partial sums) in a fixed device array
// instead of stream-ordered allocations.  For callers that cannot allocate
// (code under HIP graph capture, serving loops, harnesses that forbid it).
//
// Each device holds its own copy of the array for the life of the process.
// Host code never uses the array's name as an address: its per-device address
// comes from hipGetSymbolAddress, taken once per device on the first call with
// that device current.  Every call on a device shares that device's array, so
// calls that overlap on one device (different streams, or threads) race; the
// array keeps the last call's contents, and nothing in it needs to start at
// zero (every partial sum a call reads is written by the same call).
#include "kqr_internal.h"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace kqr {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // per device
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

// Device address of this device's array (taken once per device).
unsigned char* static_scratch() {
  int dev = 0;
  KQR_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(KQR_EINVAL, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    KQR_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(KQR_EHIP, "no device address for the static scratch array");
    g_static_ptr[dev] = p;
  }
  return static_cast<unsigned char*>(g_static_ptr[dev]);
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

// u = K v (stride incv / incu) through the fixed array.  The launch shape is
// the one kqr_kernel_apply uses, with its column segments capped so that the
// partial sums fit: the segments only split each row's sum into pieces added
// in a fixed order, so the cap changes at most that order.
void kapply_static(const KMat& km, int64_t n, const double* v, int64_t incv, double* u, int64_t incu, bool exact,
                   hipStream_t st) {
  const size_t v64_bytes = round256(size_t(n) * sizeof(double));
  const size_t v32_bytes = round256(size_t(n) * sizeof(float));
  if (v64_bytes + v32_bytes + size_t(n) * sizeof(double) > kStaticScratchBytes)
    fail(KQR_EINVAL, "n = %lld needs more than the %zu bytes of the static scratch array", (long long)n,
         kStaticScratchBytes);
  unsigned char* base = static_scratch();
  double* v64 = reinterpret_cast<double*>(base);
  float* v32 = reinterpret_cast<float*>(base + v64_bytes);
  double* part = reinterpret_cast<double*>(base + v64_bytes + v32_bytes);
  const size_t part_doubles = (kStaticScratchBytes - v64_bytes - v32_bytes) / sizeof(double);
  ApplyShape s = default_apply_shape(km.dtype, exact ? 1 : 0, n);
  s.segs = int(std::max<int64_t>(1, std::min<int64_t>(s.segs, int64_t(part_doubles / size_t(n)))));
  if (exact) {
    const double* col = v;
    if (incv != 1 || (reinterpret_cast<uintptr_t>(v) & 15) != 0) {  // the kernel reads 16-byte pieces of v
      KQR_CHECK_HIP(hipMemcpy2DAsync(v64, sizeof(double), v, size_t(incv) * sizeof(double), sizeof(double),
                                     size_t(n), hipMemcpyDeviceToDevice, st));
      col = v64;
    }
    kapply_dense(km, n, n, nullptr, col, u, incu, true, st, &s, part, part_doubles);
  } else {
    to_f32(v, n, 1, incv, v32, 1, st);
    kapply_dense(km, n, n, v32, nullptr, u, incu, false, st, &s, part, part_doubles);
  }
}

}  // namespace kqr
