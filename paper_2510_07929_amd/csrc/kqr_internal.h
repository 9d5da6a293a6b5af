// Internal declarations shared by the libkqr translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "kqr.h"

namespace kqr {

// ----------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void set_last_error(const std::string& msg);
[[noreturn]] void fail(int status, const char* fmt, ...);

#define KQR_CHECK_HIP(call)                                                         \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      ::kqr::fail(e_ == hipErrorOutOfMemory ? KQR_ENOMEM : KQR_EHIP, "%s:%d %s: %s", \
                  __FILE__, __LINE__, #call, hipGetErrorString(e_));                \
  } while (0)

#define KQR_LAUNCH_CHECK() KQR_CHECK_HIP(hipGetLastError())

// ----------------------------------------------------------------- device memory
// Owning device buffer (hipMalloc / hipFree).
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); ptr = o.ptr; bytes = o.bytes; o.ptr = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b);
  void release();
  template <typename T> T* as() const { return static_cast<T*>(ptr); }
};

// While alive on a thread, DevBuf releases on that thread are collected and
// freed when the scope ends (hipFree synchronises the device).
class DeferFrees {
 public:
  DeferFrees();
  ~DeferFrees();
  DeferFrees(const DeferFrees&) = delete;
  DeferFrees& operator=(const DeferFrees&) = delete;
  // Moves the collected pointers to out (freed by its owner instead).
  void hand_to(std::vector<void*>& out);

 private:
  std::vector<void*> list_;
  std::vector<void*>* prev_;
};

// Pinned host staging for small device->host reads.
struct HostPinned {
  void* ptr = nullptr;
  explicit HostPinned(size_t b);
  ~HostPinned();
  HostPinned(const HostPinned&) = delete;
  HostPinned& operator=(const HostPinned&) = delete;
  template <typename T> T* as() const { return static_cast<T*>(ptr); }
};

void ensure_device();  // throws KQR_ENODEVICE when no device is usable

// ----------------------------------------------------------------- kernel matrix ops
struct KernelSpec {
  int kind;      // KQR_RBF / KQR_LAPLACIAN / KQR_LINEAR
  double gamma;
};

// Materialised operator description.
struct KMat {
  const void* K = nullptr;  // nullptr: on the fly
  int dtype = KQR_FP32;
  int64_t ld = 0;           // layout 0: row stride; layout 1: tiles per side
  int layout = 0;           // 0: n x ld row-major; 1: upper-triangle tiles (kpacked.hip)
};

// Tile shape of the materialised K-apply: rows per wave, 16-byte chunks per
// lane per step, column segments per row.
struct ApplyShape {
  int rows = 8;
  int unroll = 2;
  int segs = 1;
};
ApplyShape default_apply_shape(int dtype, int exact, int64_t n);
void set_apply_shape(int dtype, int exact, int64_t n, ApplyShape s);  // autotuner override
bool apply_shape_supported(const ApplyShape& s);

// K build: K[i, j] for i < n, j < ldk (j >= n written as 0).
void kbuild(const float* X, const float* sqn, int64_t n, int p, KernelSpec ks, int dtype, void* K,
            int64_t ldk, hipStream_t st);
// K build with the Gram term on the matrix cores (RBF, p <= 32; layout 0:
// n x ldk rows, ldk a multiple of 16; layout 1: upper-triangle tiles).
// Returns false, doing nothing, for the cases it does not cover.
bool kbuild_mfma(const float* X, const float* q, int64_t n, int p, KernelSpec ks, int dtype, void* K, int64_t ldk,
                 int layout, hipStream_t st);
// Squared row norms of X (FP32).
void row_sqnorms(const float* X, int64_t n, int p, float* sqn, hipStream_t st);

// u = K v (materialised, rows [0, nrows), cols [0, ncols)).  exact: v64 + FP64; else v32.
// scratch (scratch_doubles long, or null) holds the partial sums when it is
// large enough (kapply_scratch_doubles); otherwise they are allocated on st.
void kapply_dense(const KMat& km, int64_t nrows, int64_t ncols, const float* v32, const double* v64,
                  double* u, int64_t ldu, bool exact, hipStream_t st, const ApplyShape* shape = nullptr,
                  double* scratch = nullptr, size_t scratch_doubles = 0);
// Doubles of scratch that cover every launch shape of kapply_dense on an n x n K.
size_t kapply_scratch_doubles(const KMat& km, int64_t n);
// u = shift + scale K(Xr, Xc) v computed on the fly from FP32 entries.
// exact = false: v rounded to FP32, FP32 products summed in FP32 over tiles
// of 64 columns, FP64 across tiles; exact = true: FP64 v, products and sums.
// The square apply K(X, X) v (Xr == Xc, scale 1, shift 0) of the RBF with
// p <= 32 evaluates each distinct pair once; its partial sums go to
// scratch when that holds otf_sym_scratch_doubles(n) doubles.
void kapply_otf(const float* Xr, const float* sqr, int64_t nr, const float* Xc, const float* sqc,
                int64_t nc, int p, KernelSpec ks, const double* v64, double* u, int64_t ldu,
                double out_scale, double out_shift, hipStream_t st, bool exact = false, double* scratch = nullptr,
                size_t scratch_doubles = 0);
// Laplacian on the fly from fixed-point coordinates (exact integer L1
// distances, one v_sad_u32 per coordinate).  quantize_columns fills Xq
// (n x p, stride p) with round((x - min_k) 2^s) and returns s (or -1 when X
// holds non-finite values); kapply_otf_l1q applies K(X, X) with entries
// exp(-gamma 2^-s d), each distinct pair evaluated once.  Its partial sums go
// to scratch when that holds otf_sym_scratch_doubles(n) doubles, else to
// memory allocated on st.
int quantize_columns(const float* X, int64_t n, int p, uint32_t* Xq, hipStream_t st);
size_t otf_sym_scratch_doubles(int64_t n);  // partial sums of a symmetric on-the-fly apply (0: too large)
void set_otf_sym_budget(int64_t bytes);     // largest such buffer; beyond it the row-streamed forms run
// Launch shape of the on-the-fly applies: strip = tiles per workgroup of the
// symmetric square applies (0: by size), wgs = workgroups a sliced
// rectangular launch aims for (0: 8192).
void set_otf_shape(int strip, int64_t wgs);
void set_otf_strip_for(int64_t n, int strip);  // the strip for n's size class only (0: by size)
int otf_strip_for(int64_t n);                  // the strip the symmetric applies use at n
int64_t otf_wgs();
void set_otf_wgs(int64_t wgs);  // 0: 8192

// Launch-shape registry: every shape installed by an autotuner or a
// kqr_set_* call, as the entries of the tuning file (kqr_tune_save /
// kqr_tune_load; tune.hip).  kind: "apply", "kv", "packed", "otf".
struct TuneEntry {
  std::string kind;
  int k_dtype = 0, mode = 0;
  int64_t n = 0;       // problem size the shape was chosen at (selects the size class)
  int m = 1;           // right-hand sides of the timed launch
  int a = 0, b = 0, c = 0;  // apply: rows, unroll, segs; kv: nld, prefetch, segs; packed: map, strip; otf: strip, -, -
  int64_t wgs = 0;     // otf: target workgroups of sliced launches
  double us = 0.0;     // measured launch time (0: installed by hand)
};
void tune_record(const TuneEntry& e);
int tune_save(const char* path);  // entries written
int tune_load(const char* path);  // entries installed (0 when the file was tuned on another architecture)
void tune_autoload();  // once per process: the file named by KQR_TUNE_FILE, if set
void kapply_otf_l1q(const uint32_t* Xq, int64_t n, int p, double gamma, int shift, const double* v, double* u,
                    int64_t ldu, bool exact, hipStream_t st, double* scratch = nullptr, size_t scratch_doubles = 0);
// y = A x for a skinny FP32 matrix A (nrows x ncols, ncols <= 1024, lda a
// multiple of 4) and FP64 x, y; FP64 products and sums.
void gemv_skinny(const float* A, int64_t lda, int64_t nrows, int64_t ncols, const double* x, double* y,
                 hipStream_t st);
// One row of K: out[j] = k(x_s, x_j) in FP64 (from a materialised row or from X).
void kernel_row(const KMat& km, const float* X, const float* sqn, int64_t n, int p, KernelSpec ks,
                int64_t s, double* out, hipStream_t st);

// Symmetric K as upper-triangle tiles (layout 1, tile side kPkT = 128).
int64_t packed_tile_count(int64_t n);
size_t packed_bytes(int64_t n, int dtype);
int64_t packed_tiles_per_side(int64_t n);
void kbuild_packed(const float* X, const float* sqn, int64_t n, int p, KernelSpec ks, int dtype, void* K,
                   hipStream_t st);
// Doubles of scratch kapply_packed needs (strip partials + column partials).
size_t packed_scratch_doubles(int64_t n, int strip);
// u[i ldu] = the strip partials of i's tile-row (rowpart: nt x ceil(nt/strip)
// x kPkT) plus the column partials of the tiles above i's diagonal tile
// (colpart: one kPkT-vector per upper-triangle tile), in a fixed order.
void packed_reduce(const double* rowpart, const double* colpart, int64_t n, int strip, double* u, int64_t ldu,
                   hipStream_t st);
// Launch shape of the packed K-apply: thread map (0 rows / 256 threads,
// 1 columns, 2 rows / 512 threads, 3 = 2 on a persistent grid; 4 and 5 =
// square blocks of strip x strip tiles, strip 2 or 4, each wave 32 columns
// of a tile (4) or 64 columns of half its rows (5)) and tiles per strip.
constexpr int kPkMaxStrip = 32;
struct PackedShape {
  int map = 2;
  int strip = 4;
};
// Doubles of scratch kapply_packed needs for shape s.
size_t packed_shape_scratch_doubles(int64_t n, const PackedShape& s);
PackedShape default_packed_shape(int dtype, int exact);  // tuned when set, else the fastest at n = 50,000
void set_packed_shape(int dtype, int exact, PackedShape s);
bool packed_shape_supported(const PackedShape& s);
// u = K v with K in layout 1 (n x n); scratch may be null (then allocated on st).
void kapply_packed(const KMat& km, int64_t n, const float* v32, const double* v64, double* u, int64_t ldu,
                   bool exact, hipStream_t st, const PackedShape* shape = nullptr, double* scratch = nullptr);
void kernel_row_packed(const KMat& km, int64_t n, int64_t s, double* out, hipStream_t st);

// Linear kernel k(x, x') = x^T x' in factored form (klinear.hip).  scratch:
// lin_scratch_doubles(p) doubles.
size_t lin_scratch_doubles(int p);
void lin_apply(const float* X, int64_t n, int p, const double* v, double* u, int64_t ldu, double* scratch,
               hipStream_t st);
// f = shift + scale * Xnew (Xtr^T alpha)
void lin_predict(const float* Xtr, int64_t n, int p, const double* alpha, const float* Xnew, int64_t m, double scale,
                 double shift, double* f, double* scratch, hipStream_t st);
// F = X padded to ldf columns (the exact factor of X X^T)
void lin_factor(const float* X, int64_t n, int p, float* F, int64_t ldf, hipStream_t st);

// u = K v for a materialised K (full layout) through the fixed per-device
// scratch array of kstatic.hip: no allocation (kqr_kernel_apply_static).
void kapply_static(const KMat& km, int64_t n, const double* v, int64_t incv, double* u, int64_t incu, bool exact,
                   hipStream_t st);
size_t static_scratch_bytes();

// FP64 -> FP32 copy (for the fast apply), strided rows.
void to_f32(const double* src, int64_t n, int m, int64_t lds, float* dst, int64_t ldd, hipStream_t st);

// ----------------------------------------------------------------- reductions
// Deterministic two-pass sums: kernels write per-block partials, finalize sums
// them in a fixed order into `out`.
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;
void reduce_finalize(const double* partials, int nblocks, int nq, double* out, hipStream_t st);

}  // namespace kqr
