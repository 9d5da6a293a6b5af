// Kernel-matrix operators on gfx950: materialisation, the HBM-streamed
// K-apply, the on-the-fly K-apply and single kernel rows.
//
// K_ij = exp(-gamma d_ij) with d the squared Euclidean distance (RBF) or the
// L1 distance (Laplacian) (Section 1).  exp is evaluated as exp2 of
// -gamma log2(e) d on the transcendental unit (kexp2).
#include "kernel_entry.h"
#include "kqr_internal.h"
#include "pstep.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

namespace kqr {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
// Round to nearest even (entries are finite).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// ================================================================= row norms
__global__ void sqnorm_kernel(const float* __restrict__ X, int64_t n, int p, float* __restrict__ q) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* x = X + i * p;
  float s = 0.f;
  for (int k = 0; k < p; ++k) s = fmaf(x[k], x[k], s);
  q[i] = s;
}

void row_sqnorms(const float* X, int64_t n, int p, float* sqn, hipStream_t st) {
  if (n <= 0) return;
  sqnorm_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(X, n, p, sqn);
  KQR_LAUNCH_CHECK();
}

// ================================================================= K build
bool kbuild_mfma(const float* X, const float* q, int64_t n, int p, KernelSpec ks, int dtype, void* K, int64_t ldk,
                 int layout, hipStream_t st);  // below, with the matrix-core helpers

// Laplacian, and RBF with p > 32: entries on the VALU.
// Block: 16 rows x 256 columns.  Row tile of X and its norms staged in LDS
// (broadcast reads); each thread keeps its column x_j in registers.
template <int PMAX, bool LAP, bool BF16>
__global__ __launch_bounds__(256) void kbuild_kernel(const float* __restrict__ X,
                                                     const float* __restrict__ q, int64_t n, int p,
                                                     float ng, void* __restrict__ Kout, int64_t ldk) {
  constexpr int TR = 16;
  __shared__ float xs[TR][PMAX];
  __shared__ float qs[TR];
  const int64_t i0 = (int64_t)blockIdx.x * TR;
  const int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x;
  for (int t = threadIdx.x; t < TR * PMAX; t += 256) {
    const int r = t / PMAX, k = t % PMAX;
    const int64_t i = i0 + r;
    xs[r][k] = (i < n && k < p) ? X[i * p + k] : 0.f;
  }
  if (threadIdx.x < TR) {
    const int64_t i = i0 + threadIdx.x;
    qs[threadIdx.x] = (i < n && !LAP) ? q[i] : 0.f;
  }
  __syncthreads();
  if (j >= ldk) return;
  const bool valid = j < n;
  float xj[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) xj[k] = (valid && k < p) ? X[j * p + k] : 0.f;
  const float qj = (valid && !LAP) ? q[j] : 0.f;
  for (int r = 0; r < TR; ++r) {
    const int64_t i = i0 + r;
    if (i >= n) break;
    float val = 0.f;
    if (valid) {
      float d = pair_dist<PMAX, LAP>(xs[r], qs[r], xj, qj);
      if (i == j) d = 0.f;
      val = kexp2(ng * d);
    }
    if (BF16) {
      __builtin_nontemporal_store(f32_to_bf16(val), static_cast<uint16_t*>(Kout) + i * ldk + j);
    } else {
      __builtin_nontemporal_store(val, static_cast<float*>(Kout) + i * ldk + j);
    }
  }
}

template <int PMAX>
static void kbuild_p(const float* X, const float* q, int64_t n, int p, KernelSpec ks, int dtype,
                     void* K, int64_t ldk, hipStream_t st) {
  dim3 grid((unsigned)((n + 15) / 16), (unsigned)((ldk + 255) / 256));
  const float ng = -float(ks.gamma) * kLog2e;
  const bool lap = ks.kind == KQR_LAPLACIAN, bf = dtype == KQR_BF16;
  if (lap && bf) kbuild_kernel<PMAX, true, true><<<grid, 256, 0, st>>>(X, q, n, p, ng, K, ldk);
  else if (lap) kbuild_kernel<PMAX, true, false><<<grid, 256, 0, st>>>(X, q, n, p, ng, K, ldk);
  else if (bf) kbuild_kernel<PMAX, false, true><<<grid, 256, 0, st>>>(X, q, n, p, ng, K, ldk);
  else kbuild_kernel<PMAX, false, false><<<grid, 256, 0, st>>>(X, q, n, p, ng, K, ldk);
  KQR_LAUNCH_CHECK();
}

#define KQR_DISPATCH_P(p, FN, ...)                                   \
  do {                                                               \
    if ((p) <= 8) FN<8>(__VA_ARGS__);                                \
    else if ((p) <= 12) FN<12>(__VA_ARGS__);                         \
    else if ((p) <= 16) FN<16>(__VA_ARGS__);                         \
    else if ((p) <= 20) FN<20>(__VA_ARGS__);                         \
    else if ((p) <= 24) FN<24>(__VA_ARGS__);                         \
    else if ((p) <= 32) FN<32>(__VA_ARGS__);                         \
    else if ((p) <= 48) FN<48>(__VA_ARGS__);                         \
    else if ((p) <= 64) FN<64>(__VA_ARGS__);                         \
    else fail(KQR_EINVAL, "feature dimension p=%d exceeds 64", (p)); \
  } while (0)

void kbuild(const float* X, const float* sqn, int64_t n, int p, KernelSpec ks, int dtype, void* K,
            int64_t ldk, hipStream_t st) {
  if (n <= 0) return;
  if (kbuild_mfma(X, sqn, n, p, ks, dtype, K, ldk, 0, st)) return;  // RBF, p <= 32: Gram on the matrix cores
  KQR_DISPATCH_P(p, kbuild_p, X, sqn, n, p, ks, dtype, K, ldk, st);
}

// ================================================================= materialised K-apply
// One wave streams ROWS whole rows of K with 16-byte non-temporal loads,
// UNROLL chunks per lane per step (ROWS*UNROLL loads in flight per lane); the
// vector chunk it needs is loaded once per step and shared by the ROWS rows.
// Per-lane partial sums are reduced across the wave with shuffles, so every
// output is produced by one wave in a fixed order (deterministic).
//   fast  (EXACT=false): v in FP32, FP32 products summed in FP32 over one step
//                        and then added into FP64 accumulators.
//   exact (EXACT=true) : v in FP64, products and sums in FP64.
template <bool BF16>
__device__ __forceinline__ float kelem(const u32x4& w, int e) {
  if (BF16) {
    const uint32_t word = w[e >> 1];
    return (e & 1) ? bf16_hi(word) : bf16_lo(word);
  } else {
    return __uint_as_float(w[e]);
  }
}

// Columns can be split into gridDim.y segments (smaller work items balance the
// tail of the launch); each segment then writes a partial sum per row and
// kapply_seg_reduce adds the segments in order.
template <int ROWS, int UNROLL, bool EXACT, bool BF16>
__global__ __launch_bounds__(256) void kapply_rows_kernel(const void* __restrict__ Kp, int64_t ldk,
                                                          int64_t nrows, int64_t ncols,
                                                          const float* __restrict__ v32,
                                                          const double* __restrict__ v64,
                                                          double* __restrict__ u, int64_t ldu,
                                                          int64_t seg_chunks, double* __restrict__ part) {
  constexpr int VEC = BF16 ? 8 : 4;
  constexpr int ESZ = BF16 ? 2 : 4;
  const int lane = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * ROWS;
  if (row0 >= nrows) return;
  const u32x4* rp[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const int64_t rr = (row0 + r < nrows) ? row0 + r : nrows - 1;
    rp[r] = reinterpret_cast<const u32x4*>(static_cast<const char*>(Kp) + rr * ldk * ESZ);
  }
  const int64_t nchunk_all = ncols / VEC;
  const int64_t cbeg = int64_t(blockIdx.y) * seg_chunks;
  const int64_t nchunk = min(nchunk_all, cbeg + seg_chunks);
  const bool last_seg = blockIdx.y == gridDim.y - 1;
  double acc[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) acc[r] = 0.0;

  int64_t c = cbeg + lane;
  for (; c + 64 * (UNROLL - 1) < nchunk; c += 64 * UNROLL) {
    u32x4 kk[ROWS][UNROLL];
#pragma unroll
    for (int s = 0; s < UNROLL; ++s)
#pragma unroll
      for (int r = 0; r < ROWS; ++r) kk[r][s] = __builtin_nontemporal_load(rp[r] + c + 64 * s);
    if (EXACT) {
#pragma unroll
      for (int s = 0; s < UNROLL; ++s) {
        double vv[VEC];
        const double* vp = v64 + (c + 64 * s) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; e += 2) {
          const double2 t = *reinterpret_cast<const double2*>(vp + e);
          vv[e] = t.x;
          vv[e + 1] = t.y;
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[r] = fma(double(kelem<BF16>(kk[r][s], e)), vv[e], acc[r]);
      }
    } else {
      float a32[ROWS];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) a32[r] = 0.f;
#pragma unroll
      for (int s = 0; s < UNROLL; ++s) {
        float vv[VEC];
        const float* vp = v32 + (c + 64 * s) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; e += 4) {
          const float4 t = *reinterpret_cast<const float4*>(vp + e);
          vv[e] = t.x;
          vv[e + 1] = t.y;
          vv[e + 2] = t.z;
          vv[e + 3] = t.w;
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
          for (int e = 0; e < VEC; ++e) a32[r] = fmaf(kelem<BF16>(kk[r][s], e), vv[e], a32[r]);
      }
#pragma unroll
      for (int r = 0; r < ROWS; ++r) acc[r] += double(a32[r]);
    }
  }
  for (; c < nchunk; c += 64) {
    u32x4 kk[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) kk[r] = __builtin_nontemporal_load(rp[r] + c);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const double ve = EXACT ? v64[c * VEC + e] : double(v32[c * VEC + e]);
#pragma unroll
      for (int r = 0; r < ROWS; ++r) acc[r] = fma(double(kelem<BF16>(kk[r], e)), ve, acc[r]);
    }
  }
  // trailing columns that do not fill a 16-byte chunk (last segment)
  const int64_t col = nchunk_all * VEC + lane;
  if (last_seg && col < ncols) {
    const double ve = EXACT ? v64[col] : double(v32[col]);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const char* base = reinterpret_cast<const char*>(rp[r]);
      const float ke = BF16 ? bf16_to_f32(reinterpret_cast<const uint16_t*>(base)[col])
                            : reinterpret_cast<const float*>(base)[col];
      acc[r] = fma(double(ke), ve, acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < ROWS; ++r)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
  if (part) {
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
      if (lane == r && row0 + r < nrows) part[int64_t(blockIdx.y) * nrows + row0 + r] = acc[r];
  } else {
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
      if (lane == r && row0 + r < nrows) u[(row0 + r) * ldu] = acc[r];
  }
}

__global__ void kapply_seg_reduce(const double* __restrict__ part, int nseg, int64_t nrows,
                                  double* __restrict__ u, int64_t ldu) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= nrows) return;
  double s = 0.0;
  for (int k = 0; k < nseg; ++k) s += part[int64_t(k) * nrows + i];
  u[i * ldu] = s;
}

// ----------------------------------------------------------------- shapes
namespace {
std::mutex g_shape_mu;
// tuned shapes per [dtype][exact][size bucket]
ApplyShape g_shape[2][2][3];
bool g_shape_set[2][2][3] = {};

int size_bucket(int64_t n) { return n < 8192 ? 0 : (n < 65536 ? 1 : 2); }
}  // namespace

ApplyShape default_apply_shape(int dtype, int exact, int64_t n) {
  std::lock_guard<std::mutex> lk(g_shape_mu);
  const int d = dtype == KQR_BF16, e = exact != 0, b = size_bucket(n);
  if (g_shape_set[d][e][b]) return g_shape[d][e][b];
  ApplyShape s;
  s.rows = 8;
  s.unroll = 2;
  s.segs = n >= 16384 ? 4 : 1;  // keeps work items ~n/4 columns long on large matrices
  return s;
}

void set_apply_shape(int dtype, int exact, int64_t n, ApplyShape s) {
  std::lock_guard<std::mutex> lk(g_shape_mu);
  const int d = dtype == KQR_BF16, e = exact != 0, b = size_bucket(n);
  g_shape[d][e][b] = s;
  g_shape_set[d][e][b] = true;
}

bool apply_shape_supported(const ApplyShape& s) {
  const int key = s.rows * 100 + s.unroll;
  const bool ok = key == 201 || key == 202 || key == 204 || key == 401 || key == 402 || key == 404 ||
                  key == 801 || key == 802 || key == 804;
  return ok && s.segs >= 1 && s.segs <= 64;
}

template <int ROWS, int UNROLL>
static void kapply_rows_launch(const KMat& km, int64_t nrows, int64_t ncols, const float* v32,
                               const double* v64, double* u, int64_t ldu, bool exact, int segs,
                               hipStream_t st, double* scratch, size_t scratch_doubles) {
  const int vec = km.dtype == KQR_BF16 ? 8 : 4;
  const int64_t nchunk = ncols / vec;
  segs = int(std::max<int64_t>(1, std::min<int64_t>(segs, nchunk / 64)));
  int64_t seg_chunks = (nchunk + segs - 1) / segs;
  seg_chunks = (seg_chunks + 63) / 64 * 64;
  if (seg_chunks == 0) seg_chunks = 64;
  segs = int(std::max<int64_t>(1, (nchunk + seg_chunks - 1) / seg_chunks));
  const int64_t waves = (nrows + ROWS - 1) / ROWS;
  const dim3 grid((unsigned)((waves + 3) / 4), (unsigned)segs);
  double* part = nullptr;
  const bool own = segs > 1 && !(scratch && scratch_doubles >= size_t(segs) * size_t(nrows));
  if (segs > 1) part = scratch;
  if (own)
    KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&part), size_t(segs) * nrows * sizeof(double), st));
  const bool bf = km.dtype == KQR_BF16;
  if (exact && bf)
    kapply_rows_kernel<ROWS, UNROLL, true, true><<<grid, 256, 0, st>>>(km.K, km.ld, nrows, ncols, v32, v64, u, ldu,
                                                                        seg_chunks, part);
  else if (exact)
    kapply_rows_kernel<ROWS, UNROLL, true, false><<<grid, 256, 0, st>>>(km.K, km.ld, nrows, ncols, v32, v64, u, ldu,
                                                                         seg_chunks, part);
  else if (bf)
    kapply_rows_kernel<ROWS, UNROLL, false, true><<<grid, 256, 0, st>>>(km.K, km.ld, nrows, ncols, v32, v64, u, ldu,
                                                                         seg_chunks, part);
  else
    kapply_rows_kernel<ROWS, UNROLL, false, false><<<grid, 256, 0, st>>>(km.K, km.ld, nrows, ncols, v32, v64, u, ldu,
                                                                          seg_chunks, part);
  KQR_LAUNCH_CHECK();
  if (part) {
    kapply_seg_reduce<<<dim3((unsigned)((nrows + 255) / 256)), 256, 0, st>>>(part, segs, nrows, u, ldu);
    KQR_LAUNCH_CHECK();
    if (own) KQR_CHECK_HIP(hipFreeAsync(part, st));
  }
}

void kapply_dense(const KMat& km, int64_t nrows, int64_t ncols, const float* v32, const double* v64,
                  double* u, int64_t ldu, bool exact, hipStream_t st, const ApplyShape* shape, double* scratch,
                  size_t scratch_doubles) {
  if (nrows <= 0) return;
  if (km.layout == 1) {  // symmetric upper-triangle tiles (kpacked.hip)
    if (nrows != ncols) fail(KQR_EINVAL, "the packed layout holds square K only");
    const PackedShape ps = default_packed_shape(km.dtype, exact);
    const bool fits = scratch && scratch_doubles >= packed_shape_scratch_doubles(nrows, ps);
    kapply_packed(km, nrows, v32, v64, u, ldu, exact, st, &ps, fits ? scratch : nullptr);
    return;
  }
  const ApplyShape s = shape ? *shape : default_apply_shape(km.dtype, exact, nrows);
  const int key = s.rows * 100 + s.unroll;
  switch (key) {
    case 201: kapply_rows_launch<2, 1>(km, nrows, ncols, v32, v64, u, ldu, exact, s.segs, st, scratch, scratch_doubles); break;
    case 202: kapply_rows_launch<2, 2>(km, nrows, ncols, v32, v64, u, ldu, exact, s.segs, st, scratch, scratch_doubles); break;
    case 204: kapply_rows_launch<2, 4>(km, nrows, ncols, v32, v64, u, ldu, exact, s.segs, st, scratch, scratch_doubles); break;
    case 401: kapply_rows_launch<4, 1>(km, nrows, ncols, v32, v64, u, ldu, exact, s.segs, st, scratch, scratch_doubles); break;
    case 402: kapply_rows_launch<4, 2>(km, nrows, ncols, v32, v64, u, ldu, exact, s.segs, st, scratch, scratch_doubles); break;
    case 404: kapply_rows_launch<4, 4>(km, nrows, ncols, v32, v64, u, ldu, exact, s.segs, st, scratch, scratch_doubles); break;
    case 801: kapply_rows_launch<8, 1>(km, nrows, ncols, v32, v64, u, ldu, exact, s.segs, st, scratch, scratch_doubles); break;
    case 802: kapply_rows_launch<8, 2>(km, nrows, ncols, v32, v64, u, ldu, exact, s.segs, st, scratch, scratch_doubles); break;
    case 804: kapply_rows_launch<8, 4>(km, nrows, ncols, v32, v64, u, ldu, exact, s.segs, st, scratch, scratch_doubles); break;
    default: fail(KQR_EINVAL, "unsupported K-apply shape rows=%d unroll=%d", s.rows, s.unroll);
  }
}

// ================================================================= on-the-fly K-apply
// One thread per output row i keeps x_i (and ||x_i||^2) in registers; the
// block walks a slice of the columns in tiles of 64 staged in LDS (x_j, the
// norms and v_j, read as broadcasts) and forms k(x_i, x_j) in FP32.
//   fast  (EX=false): k * v_j accumulated in FP32 over a tile (v rounded to
//                     FP32), then into an FP64 accumulator;
//   exact (EX=true) : the FP32 entry times the FP64 v_j, FP64 products and
//                     sums (the exact operator of the residuals).
// Columns are split over gridDim.y slices so that small row counts still fill
// the chip; the slices' partial sums are added in a fixed order by a second
// kernel.
constexpr int kOtfTile = 64;

// Column slices of an on-the-fly launch: about 8192 workgroups in all (many
// rounds of the blocks the chip holds at once, so the last round is a small
// tail), each slice at least 1024 columns.  Every slice writes one partial
// per row, added in slice order by otf_reduce_kernel.
std::atomic<int64_t> g_otf_wgs{8192};  // target workgroups of a sliced launch (kqr_set_otf_shape)

static int64_t otf_slices(int64_t rblk, int64_t nc) {
  const int64_t wgs = g_otf_wgs.load();
  const int64_t want = (wgs + std::max<int64_t>(rblk, 1) - 1) / std::max<int64_t>(rblk, 1);
  return std::max<int64_t>(1, std::min<int64_t>(want, (nc + 1023) / 1024));
}

template <int PMAX, bool LAP, bool EX>
__global__ __launch_bounds__(256) void kapply_otf_kernel(
    const float* __restrict__ Xr, const float* __restrict__ qr, int64_t nr,
    const float* __restrict__ Xc, const float* __restrict__ qc, int64_t nc, int p, float ng,
    const double* __restrict__ v, int64_t cols_per_slice, double* __restrict__ part) {
  __shared__ float xs[kOtfTile][PMAX];
  __shared__ float qs[kOtfTile];
  __shared__ float vs[kOtfTile];
  __shared__ double vd[kOtfTile];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const bool row_ok = i < nr;
  float xi[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) xi[k] = (row_ok && k < p) ? Xr[i * p + k] : 0.f;
  const float qi = (row_ok && !LAP) ? qr[i] : 0.f;
  const int64_t c0 = int64_t(blockIdx.y) * cols_per_slice;
  const int64_t c1 = min(nc, c0 + cols_per_slice);
  double acc = 0.0;
  for (int64_t jb = c0; jb < c1; jb += kOtfTile) {
    const int cnt = int(min<int64_t>(kOtfTile, c1 - jb));
    __syncthreads();
    for (int t = threadIdx.x; t < kOtfTile * PMAX; t += 256) {
      const int jj = t / PMAX, k = t % PMAX;
      xs[jj][k] = (jj < cnt && k < p) ? Xc[(jb + jj) * p + k] : 0.f;
    }
    if (threadIdx.x < kOtfTile) {
      const int jj = threadIdx.x;
      qs[jj] = (jj < cnt && !LAP) ? qc[jb + jj] : 0.f;
      const double vj = jj < cnt ? v[jb + jj] : 0.0;
      if (EX) vd[jj] = vj;
      else vs[jj] = float(vj);
    }
    __syncthreads();
    if (EX) {
      for (int jj = 0; jj < cnt; ++jj) {
        const float d = pair_dist<PMAX, LAP>(xs[jj], qs[jj], xi, qi);
        acc = fma(double(kexp2(ng * d)), vd[jj], acc);
      }
    } else {
      float a32 = 0.f;
      for (int jj = 0; jj < cnt; ++jj) {
        const float d = pair_dist<PMAX, LAP>(xs[jj], qs[jj], xi, qi);
        a32 = fmaf(kexp2(ng * d), vs[jj], a32);
      }
      acc += double(a32);
    }
  }
  if (row_ok) part[int64_t(blockIdx.y) * nr + i] = acc;
}

__global__ void otf_reduce_kernel(const double* __restrict__ part, int nslice, int64_t nr, double* __restrict__ u,
                                  int64_t ldu, double out_scale, double out_shift) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= nr) return;
  double s = 0.0;
  for (int k = 0; k < nslice; ++k) s += part[int64_t(k) * nr + i];
  u[i * ldu] = out_shift + out_scale * s;
}

template <int PMAX>
static void kapply_otf_p(const float* Xr, const float* qr, int64_t nr, const float* Xc,
                         const float* qc, int64_t nc, int p, KernelSpec ks, const double* v, double* u,
                         int64_t ldu, double scale, double shift, bool exact, hipStream_t st) {
  const int64_t rblk = (nr + 255) / 256;
  int64_t nslice = otf_slices(rblk, nc);
  nslice = std::min<int64_t>(nslice, 65535);
  int64_t per = (nc + nslice - 1) / nslice;
  per = (per + kOtfTile - 1) / kOtfTile * kOtfTile;
  nslice = (nc + per - 1) / per;
  double* part = nullptr;
  KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&part), size_t(nslice) * size_t(nr) * sizeof(double), st));
  const dim3 grid((unsigned)rblk, (unsigned)nslice);
  const float ng = -float(ks.gamma) * kLog2e;
  const bool lap = ks.kind == KQR_LAPLACIAN;
  if (lap && exact) kapply_otf_kernel<PMAX, true, true><<<grid, 256, 0, st>>>(Xr, qr, nr, Xc, qc, nc, p, ng, v, per, part);
  else if (lap) kapply_otf_kernel<PMAX, true, false><<<grid, 256, 0, st>>>(Xr, qr, nr, Xc, qc, nc, p, ng, v, per, part);
  else if (exact) kapply_otf_kernel<PMAX, false, true><<<grid, 256, 0, st>>>(Xr, qr, nr, Xc, qc, nc, p, ng, v, per, part);
  else kapply_otf_kernel<PMAX, false, false><<<grid, 256, 0, st>>>(Xr, qr, nr, Xc, qc, nc, p, ng, v, per, part);
  KQR_LAUNCH_CHECK();
  otf_reduce_kernel<<<dim3((unsigned)((nr + 255) / 256)), 256, 0, st>>>(part, int(nslice), nr, u, ldu, scale, shift);
  KQR_LAUNCH_CHECK();
  KQR_CHECK_HIP(hipFreeAsync(part, st));
}

// Laplacian on the fly from fixed-point coordinates.  Column k of X is
// stored as q_ik = round((x_ik - min_k) 2^s) in 32 bits (computed in FP64, so
// the only error is that rounding, at most 2^-(s+1) per coordinate), and the
// L1 distance sum_k |q_ik - q_jk| is an exact integer formed by one
// v_sad_u32 (|a - b| + c) per coordinate, against two FP32 operations per
// coordinate in the float form; s is chosen so that the sum cannot exceed
// 2^32 - 1.  The entry is exp2(-gamma log2(e) 2^-s float(d)), the rest as in
// kapply_otf_kernel.
__device__ __forceinline__ uint32_t sad_u32(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_sad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Row-streamed form over all n^2 pairs (used when the symmetric form's
// partial sums would exceed the budget below): a workgroup owns 256 R rows and a
// slice of the columns; one partial per slice and row, added by
// otf_reduce_kernel.
template <int PMAX, int R, bool EX>
__global__ __launch_bounds__(256) void kapply_otf_l1q_kernel(const uint32_t* __restrict__ Xq, int64_t n, int p,
                                                             float ngs, const double* __restrict__ v,
                                                             int64_t cols_per_slice, double* __restrict__ part) {
  // a thread owns R rows (256 R per block), so each LDS read of x_j serves R pairs
  static_assert(PMAX % 4 == 0, "coordinates are read from LDS four at a time");
  __shared__ __align__(16) uint32_t xs[kOtfTile][PMAX];
  __shared__ float vs[kOtfTile];
  __shared__ double vd[kOtfTile];
  const int64_t i0 = int64_t(blockIdx.x) * 256 * R + threadIdx.x;
  uint32_t xi[R][PMAX];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = i0 + 256 * r;
#pragma unroll
    for (int k = 0; k < PMAX; ++k) xi[r][k] = (i < n && k < p) ? Xq[i * p + k] : 0u;
  }
  const int64_t c0 = int64_t(blockIdx.y) * cols_per_slice;
  const int64_t c1 = min(n, c0 + cols_per_slice);
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  for (int64_t jb = c0; jb < c1; jb += kOtfTile) {
    const int cnt = int(min<int64_t>(kOtfTile, c1 - jb));
    __syncthreads();
    for (int t = threadIdx.x; t < kOtfTile * PMAX; t += 256) {
      const int jj = t / PMAX, k = t % PMAX;
      xs[jj][k] = (jj < cnt && k < p) ? Xq[(jb + jj) * p + k] : 0u;
    }
    if (threadIdx.x < kOtfTile) {
      const int jj = threadIdx.x;
      const double vj = jj < cnt ? v[jb + jj] : 0.0;
      if (EX) vd[jj] = vj;
      else vs[jj] = float(vj);
    }
    __syncthreads();
    float a32[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a32[r] = 0.f;
    for (int jj = 0; jj < cnt; ++jj) {
      uint32_t d[R];
#pragma unroll
      for (int r = 0; r < R; ++r) d[r] = 0u;
      const uint4* xr = reinterpret_cast<const uint4*>(xs[jj]);  // broadcast 16-byte LDS reads
#pragma unroll
      for (int k4 = 0; k4 < PMAX / 4; ++k4) {
        const uint4 c = xr[k4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          d[r] = sad_u32(xi[r][4 * k4], c.x, d[r]);
          d[r] = sad_u32(xi[r][4 * k4 + 1], c.y, d[r]);
          d[r] = sad_u32(xi[r][4 * k4 + 2], c.z, d[r]);
          d[r] = sad_u32(xi[r][4 * k4 + 3], c.w, d[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float e = kexp2(ngs * float(d[r]));
        if (EX) acc[r] = fma(double(e), vd[jj], acc[r]);
        else a32[r] = fmaf(e, vs[jj], a32[r]);
      }
    }
    if (!EX) {
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += double(a32[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = i0 + 256 * r;
    if (i < n) part[int64_t(blockIdx.y) * n + i] = acc[r];
  }
}

template <int PMAX>
static void kapply_otf_l1q_rows_p(const uint32_t* Xq, int64_t n, int p, float ngs, const double* v, double* u,
                                  int64_t ldu, bool exact, hipStream_t st) {
  // rows per thread: 4 up to 32 coordinates, 2 beyond (registers)
  constexpr int R = PMAX <= 32 ? 4 : 2;
  const int64_t rblk = (n + 256 * R - 1) / (256 * R);
  int64_t nslice = otf_slices(rblk, n);
  nslice = std::min<int64_t>(nslice, 65535);
  int64_t per = (n + nslice - 1) / nslice;
  per = (per + kOtfTile - 1) / kOtfTile * kOtfTile;
  nslice = (n + per - 1) / per;
  double* part = nullptr;
  KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&part), size_t(nslice) * size_t(n) * sizeof(double), st));
  const dim3 grid((unsigned)rblk, (unsigned)nslice);
  if (exact) kapply_otf_l1q_kernel<PMAX, R, true><<<grid, 256, 0, st>>>(Xq, n, p, ngs, v, per, part);
  else kapply_otf_l1q_kernel<PMAX, R, false><<<grid, 256, 0, st>>>(Xq, n, p, ngs, v, per, part);
  KQR_LAUNCH_CHECK();
  otf_reduce_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, st>>>(part, int(nslice), n, u, ldu, 1.0, 0.0);
  KQR_LAUNCH_CHECK();
  KQR_CHECK_HIP(hipFreeAsync(part, st));
}


// K is symmetric (Section 1), so each pair is evaluated once: over the
// upper-triangle tiles of kPkT x kPkT entries of the packed geometry.
// Workgroup b takes strip k of tile-row I (pk_strip_coords), the tiles
// J = I + k strip, ... of that row.  Thread t owns the four rows
// I kPkT + t % 32 + 32 r (fixed-point coordinates in registers, v_i) and in
// every tile the sixteen columns t / 32 + 8 c, so the two column groups of a
// wave read adjacent LDS rows (distinct banks) and every 16-byte read of
// x_j serves four pairs.  Per pair: the distance (one v_sad_u32 per
// coordinate), the entry, its product with v_j into the row sum and, off
// the diagonal tile, with v_i into the column sum.  Row sums stay in
// registers over the strip and are added over the eight column groups at its
// end (one partial per strip and row); the column sums of a tile are added
// over the 32 row groups in LDS (one partial per tile and column); a
// diagonal tile feeds its rows only.  packed_reduce adds the partials in a
// fixed order.  Fast: FP32 products and sums within a tile, FP64 beyond;
// exact: FP64 products and sums.
template <int PMAX, bool EX>
__global__ __launch_bounds__(256) void kapply_otf_l1q_sym_kernel(const uint32_t* __restrict__ Xq, int64_t n, int p,
                                                                 float ngs, const double* __restrict__ v, int64_t nt,
                                                                 int strip, int64_t nsx, double* __restrict__ rowpart,
                                                                 double* __restrict__ colpart) {
  static_assert(PMAX % 4 == 0, "coordinates are read from LDS four at a time");
  constexpr int T = kPkT;
  constexpr int R = 4;     // rows per thread
  constexpr int RG = 32;   // row groups: T / R
  constexpr int CPT = 16;  // columns per thread and tile: T / (256 / RG)
  __shared__ __align__(16) uint32_t xs[T][PMAX];
  __shared__ double vs[T];
  __shared__ double red[RG][T + 1];
  const int t = threadIdx.x;
  const int rg = t & (RG - 1), cg = t >> 5;
  int64_t I, k;
  pk_strip_coords(blockIdx.x, nt, strip, I, k);
  const int64_t J0 = I + k * strip, J1 = min(nt, J0 + strip);
  // Rows past n keep the coordinates of row n - 1 and v_i = 0: their row sums
  // are never read and their column contributions vanish.  Every load is
  // issued before any is used (a load whose use is conditional per lane would
  // be moved under the condition and waited for one at a time).
  uint32_t xi[R][PMAX];
  double vi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t ic = min(I * T + rg + RG * r, n - 1);
#pragma unroll
    for (int kk = 0; kk < PMAX; ++kk) xi[r][kk] = Xq[ic * p + min(kk, p - 1)];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = I * T + rg + RG * r;
    const double vv = v[min(i, n - 1)];
    vi[r] = i < n ? vv : 0.0;
#pragma unroll
    for (int kk = 0; kk < PMAX; ++kk) xi[r][kk] = kk < p ? xi[r][kk] : 0u;  // padded coordinates: 0 on both sides
  }
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  // The next tile's columns (coordinates of column n - 1 past n, v_j = 0
  // there) are loaded into registers while the current tile is evaluated.
  uint32_t xc[T * PMAX / 256];
  double vc = 0.0;
  auto load_cols = [&](int64_t J) {
#pragma unroll
    for (int q = 0; q < T * PMAX / 256; ++q) {
      const int e = t + 256 * q;
      const int jj = e / PMAX, kk = e % PMAX;
      xc[q] = Xq[min(J * T + jj, n - 1) * p + min(kk, p - 1)];
    }
    if (t < T) vc = v[min(J * T + t, n - 1)];
  };
  load_cols(J0);
  for (int64_t J = J0; J < J1; ++J) {
    const bool diag = J == I;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < T * PMAX / 256; ++q) {
      const int e = t + 256 * q;
      const int jj = e / PMAX, kk = e % PMAX;
      xs[jj][kk] = kk < p ? xc[q] : 0u;
    }
    if (t < T) vs[t] = J * T + t < n ? vc : 0.0;
    __syncthreads();
    if (J + 1 < J1) load_cols(J + 1);
    float a32[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a32[r] = 0.f;
#pragma unroll 2
    for (int c = 0; c < CPT; ++c) {
      const int jj = cg + 8 * c;
      uint32_t d[R];
#pragma unroll
      for (int r = 0; r < R; ++r) d[r] = 0u;
      const uint4* xr = reinterpret_cast<const uint4*>(xs[jj]);  // 16-byte LDS reads, two rows per wave
#pragma unroll
      for (int k4 = 0; k4 < PMAX / 4; ++k4) {
        const uint4 cc = xr[k4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          d[r] = sad_u32(xi[r][4 * k4], cc.x, d[r]);
          d[r] = sad_u32(xi[r][4 * k4 + 1], cc.y, d[r]);
          d[r] = sad_u32(xi[r][4 * k4 + 2], cc.z, d[r]);
          d[r] = sad_u32(xi[r][4 * k4 + 3], cc.w, d[r]);
        }
      }
      float e[R];
#pragma unroll
      for (int r = 0; r < R; ++r) e[r] = kexp2(ngs * float(d[r]));
      const double vj = vs[jj];
      if (EX) {
        double cs = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          acc[r] = fma(double(e[r]), vj, acc[r]);
          cs = fma(double(e[r]), vi[r], cs);
        }
        if (!diag) red[rg][jj] = cs;
      } else {
        float cs = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          a32[r] = fmaf(e[r], float(vj), a32[r]);
          cs = fmaf(e[r], float(vi[r]), cs);
        }
        if (!diag) red[rg][jj] = double(cs);
      }
    }
    if (!EX) {
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += double(a32[r]);
    }
    if (!diag) {  // the same in every thread of the block
      __syncthreads();
      if (t < T) {
        double cs = 0.0;
#pragma unroll 8
        for (int g = 0; g < RG; ++g) cs += red[g][t];
        colpart[size_t(pk_tile_index(I, J, nt)) * T + t] = cs;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) red[cg][rg + RG * r] = acc[r];
  __syncthreads();
  if (t < T) {
    double rs = 0.0;
#pragma unroll
    for (int g = 0; g < 256 / RG; ++g) rs += red[g][t];
    rowpart[(size_t(I) * nsx + k) * T + t] = rs;
  }
}

// Tiles per workgroup of the symmetric applies, per size class of n (tile
// rows below 64, 256, 1024, and from 1024): installed by kqr_set_otf_shape
// or the on-the-fly autotuner (1..kPkMaxStrip), else by size.
std::atomic<int> g_otf_strip[4] = {{0}, {0}, {0}, {0}};

static int otf_class(int64_t n) {
  const int64_t nt = (n + kPkT - 1) / kPkT;
  return nt >= 1024 ? 3 : (nt >= 256 ? 2 : (nt >= 64 ? 1 : 0));
}

static int otf_sym_strip(int64_t n) {
  const int c = otf_class(n);
  const int s = g_otf_strip[c].load();
  if (s > 0) return s;
  static const int rule[4] = {2, 8, 16, 32};
  return rule[c];
}

void set_otf_shape(int strip, int64_t wgs) {
  for (auto& a : g_otf_strip) a.store(strip);
  g_otf_wgs.store(wgs > 0 ? wgs : 8192);
}

void set_otf_strip_for(int64_t n, int strip) { g_otf_strip[otf_class(n)].store(strip); }

int64_t otf_wgs() { return g_otf_wgs.load(); }

void set_otf_wgs(int64_t wgs) { g_otf_wgs.store(wgs > 0 ? wgs : 8192); }

int otf_strip_for(int64_t n) { return otf_sym_strip(n); }

// The symmetric applies keep one FP64 partial per tile and column, about
// n^2 / 32 bytes (3 GB at n = 300,000, 31 GB at n = 10^6).  Beyond a
// budget (32 GiB unless set) the row-streamed forms run instead (all n^2
// pairs, O(n) partials).
std::atomic<int64_t> g_otf_sym_budget{int64_t(32) << 30};

void set_otf_sym_budget(int64_t bytes) { g_otf_sym_budget.store(bytes); }

static bool otf_sym_fits(int64_t n) {
  return int64_t(packed_scratch_doubles(n, otf_sym_strip(n)) * sizeof(double)) <= g_otf_sym_budget.load();
}

size_t otf_sym_scratch_doubles(int64_t n) {
  return otf_sym_fits(n) ? packed_scratch_doubles(n, otf_sym_strip(n)) : 0;
}

template <int PMAX>
static void kapply_otf_l1q_p(const uint32_t* Xq, int64_t n, int p, float ngs, const double* v, double* u, int64_t ldu,
                             bool exact, hipStream_t st, double* scratch, size_t scratch_doubles) {
  if (!otf_sym_fits(n)) {
    kapply_otf_l1q_rows_p<PMAX>(Xq, n, p, ngs, v, u, ldu, exact, st);
    return;
  }
  const int64_t nt = (n + kPkT - 1) / kPkT;
  const int strip = otf_sym_strip(n);
  const int64_t nsx = (nt + strip - 1) / strip;
  const size_t need = packed_scratch_doubles(n, strip);
  double* buf = scratch && scratch_doubles >= need ? scratch : nullptr;
  const bool own = buf == nullptr;
  if (own) KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&buf), need * sizeof(double), st));
  double* rowpart = buf;
  double* colpart = buf + size_t(nt) * nsx * kPkT;
  const dim3 grid((unsigned)pk_strips_tail(nt, strip));
  if (exact)
    kapply_otf_l1q_sym_kernel<PMAX, true><<<grid, 256, 0, st>>>(Xq, n, p, ngs, v, nt, strip, nsx, rowpart, colpart);
  else
    kapply_otf_l1q_sym_kernel<PMAX, false><<<grid, 256, 0, st>>>(Xq, n, p, ngs, v, nt, strip, nsx, rowpart, colpart);
  KQR_LAUNCH_CHECK();
  packed_reduce(rowpart, colpart, n, strip, u, ldu, st);
  if (own) KQR_CHECK_HIP(hipFreeAsync(buf, st));
}

void kapply_otf_l1q(const uint32_t* Xq, int64_t n, int p, double gamma, int shift, const double* v, double* u,
                    int64_t ldu, bool exact, hipStream_t st, double* scratch, size_t scratch_doubles) {
  if (n <= 0) return;
  const float ngs = float(-gamma * double(kLog2e) * std::ldexp(1.0, -shift));
  KQR_DISPATCH_P(p, kapply_otf_l1q_p, Xq, n, p, ngs, v, u, ldu, exact, st, scratch, scratch_doubles);
}

// Per-column minimum and maximum of X (FP32 values, exact); mm: 2 p floats.
__global__ void col_minmax_kernel(const float* __restrict__ X, int64_t n, int p, float* __restrict__ mm) {
  const int k = blockIdx.x;
  float lo = INFINITY, hi = -INFINITY;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float x = X[i * p + k];
    lo = fminf(lo, x);
    hi = fmaxf(hi, x);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off));
    hi = fmaxf(hi, __shfl_xor(hi, off));
  }
  __shared__ float sl[4], sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sl[wave] = lo; sh[wave] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    mm[2 * k] = fminf(fminf(sl[0], sl[1]), fminf(sl[2], sl[3]));
    mm[2 * k + 1] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
  }
}

__global__ void quantize_kernel(const float* __restrict__ X, int64_t n, int p, const float* __restrict__ mm,
                                double scale, uint32_t* __restrict__ Xq) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= n * p) return;
  const int k = int(t % p);
  Xq[t] = uint32_t(llrint((double(X[t]) - double(mm[2 * k])) * scale));
}

int quantize_columns(const float* X, int64_t n, int p, uint32_t* Xq, hipStream_t st) {
  if (n <= 0 || p <= 0) return -1;
  float* mm = nullptr;
  KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&mm), size_t(2 * p) * sizeof(float), st));
  col_minmax_kernel<<<dim3((unsigned)p), 256, 0, st>>>(X, n, p, mm);
  KQR_LAUNCH_CHECK();
  std::vector<float> h(size_t(2 * p));
  KQR_CHECK_HIP(hipMemcpyAsync(h.data(), mm, h.size() * sizeof(float), hipMemcpyDeviceToHost, st));
  KQR_CHECK_HIP(hipStreamSynchronize(st));
  double range = 0.0;
  for (int k = 0; k < p; ++k) {
    const double r = double(h[size_t(2 * k + 1)]) - double(h[size_t(2 * k)]);
    if (!std::isfinite(r)) {
      KQR_CHECK_HIP(hipFreeAsync(mm, st));
      return -1;
    }
    range = std::max(range, r);
  }
  // largest s <= 23 with p * range * 2^s + p <= 2^32 - 1 (sum of rounded coordinates)
  int s = 23;
  while (s >= 0 && double(p) * (range * std::ldexp(1.0, s) + 1.0) > 4294967295.0) --s;
  if (s >= 0) {
    const int64_t tot = n * p;
    quantize_kernel<<<dim3((unsigned)((tot + 255) / 256)), 256, 0, st>>>(X, n, p, mm, std::ldexp(1.0, s), Xq);
    KQR_LAUNCH_CHECK();
  }
  KQR_CHECK_HIP(hipFreeAsync(mm, st));
  return s;
}

// RBF on the fly with the Gram term on the matrix cores: a wave owns two
// 16-row strips (its rows of X held as MFMA A operands for the whole launch),
// the block stages 64 columns of X, their norms and v in LDS, and for each
// 16-column tile v_mfma_f32_16x16x4f32 forms the 16 x 16 Gram blocks
// (KP/4 MFMAs per strip, FP32 products and sums).  The lane that holds
// G[4g + r][c] then forms d = q_i + q_j - 2 G, exp2(-gamma log2(e) d) and
// accumulates k * v_j (fast: FP32 per 64-column stage, then FP64; exact: FP64
// products and sums); the 16 lanes of a row group are reduced with shuffles
// at the end.  KP = p rounded up to 4 (<= 32).
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int kMfmaCols = 64;

template <int KP, bool EX>
__global__ __launch_bounds__(256) void kapply_otf_mfma_kernel(
    const float* __restrict__ Xr, const float* __restrict__ qr, int64_t nr,
    const float* __restrict__ Xc, const float* __restrict__ qc, int64_t nc, int p, float ng,
    const double* __restrict__ v, int64_t cols_per_slice, double* __restrict__ part) {
  constexpr int NKB = KP / 4;
  __shared__ float xs[kMfmaCols][KP + 1];
  __shared__ float qs[kMfmaCols];
  __shared__ float vs[kMfmaCols];
  __shared__ double vd[kMfmaCols];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t row0 = int64_t(blockIdx.x) * 128 + wave * 32;
  float a[2][NKB];
  float qi[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int64_t r = row0 + 16 * s + li;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      const int k = 4 * kb + lg;
      a[s][kb] = (r < nr && k < p) ? Xr[r * p + k] : 0.f;
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t ro = row0 + 16 * s + 4 * lg + rr;
      qi[s][rr] = ro < nr ? qr[ro] : 0.f;
    }
  }
  const int64_t c0 = int64_t(blockIdx.y) * cols_per_slice;
  const int64_t c1 = min(nc, c0 + cols_per_slice);
  double acc[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[s][rr] = 0.0;
  for (int64_t jb = c0; jb < c1; jb += kMfmaCols) {
    const int cnt = int(min<int64_t>(kMfmaCols, c1 - jb));
    __syncthreads();
    for (int t = threadIdx.x; t < kMfmaCols * KP; t += 256) {
      const int jj = t / KP, k = t % KP;
      xs[jj][k] = (jj < cnt && k < p) ? Xc[(jb + jj) * p + k] : 0.f;
    }
    if (threadIdx.x < kMfmaCols) {
      const int jj = threadIdx.x;
      qs[jj] = jj < cnt ? qc[jb + jj] : 0.f;
      const double vj = jj < cnt ? v[jb + jj] : 0.0;
      if (EX) vd[jj] = vj;
      else vs[jj] = float(vj);
    }
    __syncthreads();
    float a32[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) a32[s][rr] = 0.f;
    // Gram blocks of the next 16-column tile are issued to the matrix cores
    // before the current tile's exponentials, so one wave keeps both busy.
    auto gram = [&](int t16, f32x4_t& g0, f32x4_t& g1) {
      const int jj = t16 + li;
      float b[NKB];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) b[kb] = xs[jj][4 * kb + lg];
      g0 = f32x4_t{0.f, 0.f, 0.f, 0.f};
      g1 = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        g0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][kb], b[kb], g0, 0, 0, 0);
        g1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1][kb], b[kb], g1, 0, 0, 0);
      }
    };
    f32x4_t g0, g1, n0, n1;
    gram(0, g0, g1);
    for (int t16 = 0; t16 < cnt; t16 += 16) {
      const int jj = t16 + li;
      const bool more = t16 + 16 < cnt;
      if (more) gram(t16 + 16, n0, n1);
      const float qj = qs[jj];
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        // ng < 0, d >= 0: exp2(ng max(d, 0)) = min(exp2(ng d), 1), clamped by the output modifier
        const float d0 = qi[0][rr] + qj - 2.f * g0[rr];
        const float d1 = qi[1][rr] + qj - 2.f * g1[rr];
        const float e0 = __builtin_amdgcn_fmed3f(kexp2(ng * d0), 0.f, 1.f);
        const float e1 = __builtin_amdgcn_fmed3f(kexp2(ng * d1), 0.f, 1.f);
        if (EX) {
          acc[0][rr] = fma(double(e0), vd[jj], acc[0][rr]);
          acc[1][rr] = fma(double(e1), vd[jj], acc[1][rr]);
        } else {
          a32[0][rr] = fmaf(e0, vs[jj], a32[0][rr]);
          a32[1][rr] = fmaf(e1, vs[jj], a32[1][rr]);
        }
      }
      if (more) {
        g0 = n0;
        g1 = n1;
      }
    }
    if (!EX) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[s][rr] += double(a32[s][rr]);
    }
  }
  // sum over the 16 column lanes of each row group (lane bits 0..3)
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      double x = acc[s][rr];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) x += __shfl_xor(x, off);
      acc[s][rr] = x;
    }
  if (li == 0) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int64_t ro = row0 + 16 * s + 4 * lg + rr;
        if (ro < nr) part[int64_t(blockIdx.y) * nr + ro] = acc[s][rr];
      }
  }
}

// The same with the Gram term in BF16 on the matrix cores: every FP32
// coordinate is split exactly into three BF16 parts x = h + m + l (round to
// nearest even at each step; 3 x 8 significand bits hold FP32's 24), and
// G = hh + hm + mh + hl + lh + mm (the dropped ml, lm, ll are below 2^-24 of
// |x_i| |x_j| per coordinate) is formed by six v_mfma_f32_16x16x32_bf16 per
// 16 x 16 block (p <= 32, padded to 32), against eight 16x16x4 FP32 MFMAs
// that take 5x the matrix-core time at p = 32.  FP32 sums inside the MFMA.
//
// The column side is split once per launch into a buffer of three planes
// per column (kotf_split_cols_kernel).  With p <= 30 (AUG) the two spare
// coordinates carry the squared norms and the column side the exponent's
// scale c = -gamma log2(e): row [x_i, 1, q_i] against column
// [-2 c x_j, c q_j, c] (each product rounded once in FP32 before the split),
// so the matrix cores return c d_ij = c (q_i + q_j - 2 x_i . x_j) itself and
// a pair costs the lanes only the clamp at 0, the exponential and the
// product with v_j.  Without AUG the column holds -2 x_j (exact) and the
// lanes add q_i + q_j and scale.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split3_bf16(float x, uint16_t& h, uint16_t& m, uint16_t& l) {
  h = f32_to_bf16(x);
  const float r1 = x - bf16_to_f32(h);  // exact
  m = f32_to_bf16(r1);
  const float r2 = r1 - bf16_to_f32(m);  // exact, at most 8 significant bits
  l = f32_to_bf16(r2);
}

constexpr int kB3Cols = 128;   // columns per LDS stage
constexpr int kB3Row = 40;     // LDS row of 32 BF16 coordinates, padded (16-byte aligned, rows spread over banks)
constexpr int kB3Stride = 96;  // halves per column in the split buffer: the h, m and l planes of 32

// Coordinate k of the padded 32-vector of a row (A) or column (B) side;
// c: the column side's scale (AUG), else 1.
template <bool AUG, bool COL>
__device__ __forceinline__ float b3_coord(const float* __restrict__ x, float q, int k, int p, float c) {
  if (k < p) return COL ? (-2.f * c) * x[k] : x[k];
  if (AUG && k == 30) return COL ? c * q : 1.f;
  if (AUG && k == 31) return COL ? c : q;
  return 0.f;
}

// out[j * 96 + plane * 32 + k]: the parts of point j's coordinate k, as the
// column (scaled, COL) or the row side; one thread per point and
// 8-coordinate group.
template <bool AUG, bool COL = true>
__global__ __launch_bounds__(256) void kotf_split_cols_kernel(const float* __restrict__ Xc,
                                                              const float* __restrict__ qc, int64_t nc, int p,
                                                              float ng, uint16_t* __restrict__ out) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= nc * 4) return;
  const int64_t j = t >> 2;
  const int g = int(t & 3);
  const float q = AUG ? qc[j] : 0.f;
  u16x8_t h, m, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    uint16_t hh, mm, ll;
    split3_bf16(b3_coord<AUG, COL>(Xc + j * p, q, 8 * g + e, p, (AUG && COL) ? ng : 1.f), hh, mm, ll);
    h[e] = hh;
    m[e] = mm;
    l[e] = ll;
  }
  uint16_t* o = out + j * kB3Stride + 8 * g;
  *reinterpret_cast<u16x8_t*>(o) = h;
  *reinterpret_cast<u16x8_t*>(o + 32) = m;
  *reinterpret_cast<u16x8_t*>(o + 64) = l;
}

template <bool EX, bool AUG>
__global__ __launch_bounds__(256) void kapply_otf_mfma3_kernel(
    const float* __restrict__ Xr, const float* __restrict__ qr, int64_t nr, const uint16_t* __restrict__ Bc,
    const float* __restrict__ qc, int64_t nc, int p, float ng, const double* __restrict__ v,
    int64_t cols_per_slice, double* __restrict__ part) {
  __shared__ __align__(16) uint16_t bs[3][kB3Cols][kB3Row];
  __shared__ float qs[AUG ? 1 : kB3Cols];
  __shared__ float vs[kB3Cols];
  __shared__ double vd[kB3Cols];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t row0 = int64_t(blockIdx.x) * 128 + wave * 32;
  bf16x8_t ah[2], am[2], al[2];
  float qi[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int64_t r = row0 + 16 * s + li;
    const bool in = r < nr;
    const float q = (AUG && in) ? qr[r] : 0.f;
    u16x8_t h, m, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * lg + e;
      const float x = in ? b3_coord<AUG, false>(Xr + r * p, q, k, p, 1.f) : 0.f;
      uint16_t hh, mm, ll;
      split3_bf16(x, hh, mm, ll);
      h[e] = hh;
      m[e] = mm;
      l[e] = ll;
    }
    ah[s] = __builtin_bit_cast(bf16x8_t, h);
    am[s] = __builtin_bit_cast(bf16x8_t, m);
    al[s] = __builtin_bit_cast(bf16x8_t, l);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t ro = row0 + 16 * s + 4 * lg + rr;
      qi[s][rr] = (!AUG && ro < nr) ? qr[ro] : 0.f;
    }
  }
  const int64_t c0 = int64_t(blockIdx.y) * cols_per_slice;
  const int64_t c1 = min(nc, c0 + cols_per_slice);
  double acc[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[s][rr] = 0.0;
  for (int64_t jb = c0; jb < c1; jb += kB3Cols) {
    const int cnt = int(min<int64_t>(kB3Cols, c1 - jb));
    __syncthreads();
    // 16-byte chunks: column jj, plane pl, coordinates 8g..8g+7
    for (int t = threadIdx.x; t < kB3Cols * 12; t += 256) {
      const int jj = t / 12, r = t - 12 * (t / 12), pl = r >> 2, g = r & 3;
      u16x8_t val = u16x8_t{0, 0, 0, 0, 0, 0, 0, 0};
      if (jj < cnt) val = *reinterpret_cast<const u16x8_t*>(Bc + (jb + jj) * kB3Stride + 32 * pl + 8 * g);
      *reinterpret_cast<u16x8_t*>(&bs[pl][jj][8 * g]) = val;
    }
    if (threadIdx.x < kB3Cols) {
      const int jj = threadIdx.x;
      if (!AUG) qs[jj] = jj < cnt ? qc[jb + jj] : 0.f;
      const double vj = jj < cnt ? v[jb + jj] : 0.0;
      if (EX) vd[jj] = vj;
      else vs[jj] = float(vj);
    }
    __syncthreads();
    float a32[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) a32[s][rr] = 0.f;
    // Gram blocks of one 16-column tile (issuing the next tile's MFMAs ahead
    // of these exponentials measured slower: the other waves of the SIMD
    // already fill the matrix-core latency)
    auto gram = [&](int t16, f32x4_t* g) {
      const int jj = t16 + li;
      const bf16x8_t b_h = *reinterpret_cast<const bf16x8_t*>(&bs[0][jj][8 * lg]);
      const bf16x8_t b_m = *reinterpret_cast<const bf16x8_t*>(&bs[1][jj][8 * lg]);
      const bf16x8_t b_l = *reinterpret_cast<const bf16x8_t*>(&bs[2][jj][8 * lg]);
#pragma unroll
      for (int s = 0; s < 2; ++s) {  // smallest products first
        f32x4_t c = f32x4_t{0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[s], b_m, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], b_l, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[s], b_h, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], b_m, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[s], b_h, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], b_h, c, 0, 0, 0);
        g[s] = c;
      }
    };
    f32x4_t g[2];
    for (int t16 = 0; t16 < cnt; t16 += 16) {
      const int jj = t16 + li;
      gram(t16, g);
      const float qj = AUG ? 0.f : qs[jj];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          // ng < 0 and d >= 0: exp2(min(ng d, 0)) = min(exp2(ng d), 1), the clamp
          // to [0, 1] being the exponential's output modifier
          const float a = AUG ? g[s][rr] : ng * (qi[s][rr] + qj + g[s][rr]);
          const float e = __builtin_amdgcn_fmed3f(kexp2(a), 0.f, 1.f);
          if (EX) acc[s][rr] = fma(double(e), vd[jj], acc[s][rr]);
          else a32[s][rr] = fmaf(e, vs[jj], a32[s][rr]);
        }
    }
    if (!EX) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[s][rr] += double(a32[s][rr]);
    }
  }
  // sum over the 16 column lanes of each row group (lane bits 0..3)
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      double x = acc[s][rr];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) x += __shfl_xor(x, off);
      acc[s][rr] = x;
    }
  if (li == 0) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int64_t ro = row0 + 16 * s + 4 * lg + rr;
        if (ro < nr) part[int64_t(blockIdx.y) * nr + ro] = acc[s][rr];
      }
  }
}

// Symmetric form of the BF16x3 apply for the square K(X, X): each distinct
// pair once, over the upper-triangle 128 x 128 tiles of the packed geometry.
// A workgroup takes a strip of tiles of tile-row I; its rows are held as in
// kapply_otf_mfma3_kernel (wave w: rows 32 w .. 32 w + 31 of the tile-row,
// split once into registers) and each tile J is one 128-column stage.
// Every entry feeds the row sum (times v_j) and, off the diagonal tile, the
// column sum (times v_i): a lane adds its eight rows, the four lane groups
// are added across lanes and the four waves in LDS.  Row sums are added over
// the 16 column lanes at the end of the strip.  packed_reduce adds the
// partials in a fixed order.
template <bool EX, bool AUG>
__global__ __launch_bounds__(256) void kapply_otf_mfma3_sym_kernel(
    const float* __restrict__ X, const float* __restrict__ q, int64_t n, const uint16_t* __restrict__ Bc, int p,
    float ng, const double* __restrict__ v, int64_t nt, int strip, int64_t nsx, double* __restrict__ rowpart,
    double* __restrict__ colpart) {
  static_assert(kB3Cols == kPkT, "one stage per tile");
  __shared__ __align__(16) uint16_t bs[3][kB3Cols][kB3Row];
  __shared__ float qs[AUG ? 1 : kB3Cols];
  __shared__ double vd[kB3Cols];
  __shared__ double red[4][kB3Cols];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int li = lane & 15, lg = lane >> 4;
  int64_t I, kst;
  pk_strip_coords(blockIdx.x, nt, strip, I, kst);
  const int64_t J0 = I + kst * strip, J1 = min(nt, J0 + strip);
  const int64_t row0 = I * kPkT + wave * 32;
  bf16x8_t ah[2], am[2], al[2];
  float qi[2][4];
  double vi[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int64_t r = row0 + 16 * s + li;
    const bool in = r < n;
    const float qq = (AUG && in) ? q[r] : 0.f;
    u16x8_t h, m, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * lg + e;
      const float x = in ? b3_coord<AUG, false>(X + r * p, qq, k, p, 1.f) : 0.f;
      uint16_t hh, mm, ll;
      split3_bf16(x, hh, mm, ll);
      h[e] = hh;
      m[e] = mm;
      l[e] = ll;
    }
    ah[s] = __builtin_bit_cast(bf16x8_t, h);
    am[s] = __builtin_bit_cast(bf16x8_t, m);
    al[s] = __builtin_bit_cast(bf16x8_t, l);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t ro = row0 + 16 * s + 4 * lg + rr;
      const int64_t rc = min(ro, n - 1);
      const float qv = q[rc];
      const double vv = v[rc];
      qi[s][rr] = (!AUG && ro < n) ? qv : 0.f;
      vi[s][rr] = ro < n ? vv : 0.0;  // rows past n add nothing to the column sums
    }
  }
  double acc[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[s][rr] = 0.0;
  for (int64_t J = J0; J < J1; ++J) {
    const bool diag = J == I;
    const int64_t jb = J * kPkT;
    const int cnt = int(min<int64_t>(kB3Cols, n - jb));
    __syncthreads();
    for (int e = t; e < kB3Cols * 12; e += 256) {
      const int jj = e / 12, r = e - 12 * (e / 12), pl = r >> 2, g = r & 3;
      u16x8_t val = u16x8_t{0, 0, 0, 0, 0, 0, 0, 0};
      if (jj < cnt) val = *reinterpret_cast<const u16x8_t*>(Bc + (jb + jj) * kB3Stride + 32 * pl + 8 * g);
      *reinterpret_cast<u16x8_t*>(&bs[pl][jj][8 * g]) = val;
    }
    if (t < kB3Cols) {
      if (!AUG) qs[t] = t < cnt ? q[jb + t] : 0.f;
      vd[t] = t < cnt ? v[jb + t] : 0.0;
    }
    __syncthreads();
    float a32[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) a32[s][rr] = 0.f;
    for (int t16 = 0; t16 < cnt; t16 += 16) {
      const int jj = t16 + li;
      const bf16x8_t b_h = *reinterpret_cast<const bf16x8_t*>(&bs[0][jj][8 * lg]);
      const bf16x8_t b_m = *reinterpret_cast<const bf16x8_t*>(&bs[1][jj][8 * lg]);
      const bf16x8_t b_l = *reinterpret_cast<const bf16x8_t*>(&bs[2][jj][8 * lg]);
      f32x4_t g[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {  // smallest products first
        f32x4_t c = f32x4_t{0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[s], b_m, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], b_l, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[s], b_h, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], b_m, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[s], b_h, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], b_h, c, 0, 0, 0);
        g[s] = c;
      }
      const float qj = AUG ? 0.f : qs[jj];
      const double vj = vd[jj];
      double cs64 = 0.0;
      float cs32 = 0.f;
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          // ng < 0 and d >= 0: exp2(min(ng d, 0)) = min(exp2(ng d), 1), the clamp
          // to [0, 1] being the exponential's output modifier
          const float a = AUG ? g[s][rr] : ng * (qi[s][rr] + qj + g[s][rr]);
          const float e = __builtin_amdgcn_fmed3f(kexp2(a), 0.f, 1.f);
          if (EX) {
            acc[s][rr] = fma(double(e), vj, acc[s][rr]);
            cs64 = fma(double(e), vi[s][rr], cs64);
          } else {
            a32[s][rr] = fmaf(e, float(vj), a32[s][rr]);
            cs32 = fmaf(e, float(vi[s][rr]), cs32);
          }
        }
      if (!diag) {  // the column's 32 rows of this wave: add the four lane groups
        double cs = EX ? cs64 : double(cs32);
        cs += __shfl_xor(cs, 16);
        cs += __shfl_xor(cs, 32);
        if (lg == 0) red[wave][jj] = cs;
      }
    }
    if (!EX) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[s][rr] += double(a32[s][rr]);
    }
    if (!diag) {  // the same in every thread of the block
      __syncthreads();
      if (t < kB3Cols)
        colpart[size_t(pk_tile_index(I, J, nt)) * kPkT + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    }
  }
  // row sums over the 16 column lanes of each row group (lane bits 0..3)
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      double x = acc[s][rr];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) x += __shfl_xor(x, off);
      acc[s][rr] = x;
    }
  if (li == 0) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        rowpart[(size_t(I) * nsx + kst) * kPkT + wave * 32 + 16 * s + 4 * lg + rr] = acc[s][rr];
  }
}

// The same for p <= 16 with the Gram term on v_mfma_f32_16x16x4f32 (FP32
// operands, as kapply_otf_mfma_kernel): each distinct pair of the square
// K(X, X) once, in the strip and tile geometry above.
template <int KP, bool EX>
__global__ __launch_bounds__(256) void kapply_otf_mfma_sym_kernel(
    const float* __restrict__ X, const float* __restrict__ q, int64_t n, int p, float ng,
    const double* __restrict__ v, int64_t nt, int strip, int64_t nsx, double* __restrict__ rowpart,
    double* __restrict__ colpart) {
  constexpr int NKB = KP / 4;
  constexpr int T = kPkT;
  __shared__ float xs[T][KP + 1];
  __shared__ float qs[T];
  __shared__ double vd[T];
  __shared__ double red[4][T];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int li = lane & 15, lg = lane >> 4;
  int64_t I, kst;
  pk_strip_coords(blockIdx.x, nt, strip, I, kst);
  const int64_t J0 = I + kst * strip, J1 = min(nt, J0 + strip);
  const int64_t row0 = I * T + wave * 32;
  float a[2][NKB];
  float qi[2][4];
  double vi[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int64_t r = row0 + 16 * s + li;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      const int k = 4 * kb + lg;
      a[s][kb] = (r < n && k < p) ? X[r * p + k] : 0.f;
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t ro = row0 + 16 * s + 4 * lg + rr;
      const int64_t rc = min(ro, n - 1);
      const float qv = q[rc];
      const double vv = v[rc];
      qi[s][rr] = ro < n ? qv : 0.f;
      vi[s][rr] = ro < n ? vv : 0.0;  // rows past n add nothing to the column sums
    }
  }
  double acc[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[s][rr] = 0.0;
  for (int64_t J = J0; J < J1; ++J) {
    const bool diag = J == I;
    const int64_t jb = J * T;
    const int cnt = int(min<int64_t>(T, n - jb));
    __syncthreads();
    for (int e = t; e < T * KP; e += 256) {
      const int jj = e / KP, k = e % KP;
      xs[jj][k] = (jj < cnt && k < p) ? X[(jb + jj) * p + k] : 0.f;
    }
    if (t < T) {
      qs[t] = t < cnt ? q[jb + t] : 0.f;
      vd[t] = t < cnt ? v[jb + t] : 0.0;
    }
    __syncthreads();
    float a32[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) a32[s][rr] = 0.f;
    for (int t16 = 0; t16 < cnt; t16 += 16) {
      const int jj = t16 + li;
      float b[NKB];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) b[kb] = xs[jj][4 * kb + lg];
      f32x4_t g0 = f32x4_t{0.f, 0.f, 0.f, 0.f}, g1 = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        g0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][kb], b[kb], g0, 0, 0, 0);
        g1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1][kb], b[kb], g1, 0, 0, 0);
      }
      const float qj = qs[jj];
      const double vj = vd[jj];
      double cs64 = 0.0;
      float cs32 = 0.f;
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const float gg = s == 0 ? g0[rr] : g1[rr];
          // ng < 0, d >= 0: exp2(ng max(d, 0)) = min(exp2(ng d), 1), clamped by the output modifier
          const float e = __builtin_amdgcn_fmed3f(kexp2(ng * (qi[s][rr] + qj - 2.f * gg)), 0.f, 1.f);
          if (EX) {
            acc[s][rr] = fma(double(e), vj, acc[s][rr]);
            cs64 = fma(double(e), vi[s][rr], cs64);
          } else {
            a32[s][rr] = fmaf(e, float(vj), a32[s][rr]);
            cs32 = fmaf(e, float(vi[s][rr]), cs32);
          }
        }
      if (!diag) {  // the column's 32 rows of this wave: add the four lane groups
        double cs = EX ? cs64 : double(cs32);
        cs += __shfl_xor(cs, 16);
        cs += __shfl_xor(cs, 32);
        if (lg == 0) red[wave][jj] = cs;
      }
    }
    if (!EX) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[s][rr] += double(a32[s][rr]);
    }
    if (!diag) {  // the same in every thread of the block
      __syncthreads();
      if (t < T) colpart[size_t(pk_tile_index(I, J, nt)) * T + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      double x = acc[s][rr];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) x += __shfl_xor(x, off);
      acc[s][rr] = x;
    }
  if (li == 0) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        rowpart[(size_t(I) * nsx + kst) * T + wave * 32 + 16 * s + 4 * lg + rr] = acc[s][rr];
  }
}

// K(X, X) v with each distinct pair once (RBF, p <= 32; KP = p rounded up to
// 4, the BF16x3 Gram above 16); u = K v.
template <int KP>
static void kapply_otf_mfma_sym(const float* X, const float* q, int64_t n, int p, KernelSpec ks, const double* v,
                                double* u, int64_t ldu, bool exact, hipStream_t st, double* scratch,
                                size_t scratch_doubles) {
  const int64_t nt = (n + kPkT - 1) / kPkT;
  const int strip = otf_sym_strip(n);
  const int64_t nsx = (nt + strip - 1) / strip;
  const size_t need = packed_scratch_doubles(n, strip);
  const size_t split_bytes = KP > 16 ? size_t(n) * kB3Stride * sizeof(uint16_t) : 0;
  double* part = scratch && scratch_doubles >= need ? scratch : nullptr;
  const size_t part_bytes = part ? 0 : (need * sizeof(double) + 255) / 256 * 256;
  char* buf = nullptr;
  if (part_bytes + split_bytes > 0)
    KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&buf), part_bytes + split_bytes, st));
  if (!part) part = reinterpret_cast<double*>(buf);
  double* rowpart = part;
  double* colpart = part + size_t(nt) * nsx * kPkT;
  const float ng = -float(ks.gamma) * kLog2e;
  const dim3 grid((unsigned)pk_strips_tail(nt, strip));
  if (KP <= 16) {
    if (exact)
      kapply_otf_mfma_sym_kernel<KP, true><<<grid, 256, 0, st>>>(X, q, n, p, ng, v, nt, strip, nsx, rowpart, colpart);
    else
      kapply_otf_mfma_sym_kernel<KP, false><<<grid, 256, 0, st>>>(X, q, n, p, ng, v, nt, strip, nsx, rowpart, colpart);
    KQR_LAUNCH_CHECK();
    packed_reduce(rowpart, colpart, n, strip, u, ldu, st);
    if (buf) KQR_CHECK_HIP(hipFreeAsync(buf, st));
    return;
  }
  uint16_t* bc = reinterpret_cast<uint16_t*>(buf + part_bytes);
  const bool aug = p <= 30;
  const dim3 sgrid((unsigned)((n * 4 + 255) / 256));
  if (aug) kotf_split_cols_kernel<true><<<sgrid, 256, 0, st>>>(X, q, n, p, ng, bc);
  else kotf_split_cols_kernel<false><<<sgrid, 256, 0, st>>>(X, q, n, p, ng, bc);
  KQR_LAUNCH_CHECK();
  if (aug && exact)
    kapply_otf_mfma3_sym_kernel<true, true><<<grid, 256, 0, st>>>(X, q, n, bc, p, ng, v, nt, strip, nsx, rowpart, colpart);
  else if (aug)
    kapply_otf_mfma3_sym_kernel<false, true><<<grid, 256, 0, st>>>(X, q, n, bc, p, ng, v, nt, strip, nsx, rowpart, colpart);
  else if (exact)
    kapply_otf_mfma3_sym_kernel<true, false><<<grid, 256, 0, st>>>(X, q, n, bc, p, ng, v, nt, strip, nsx, rowpart, colpart);
  else
    kapply_otf_mfma3_sym_kernel<false, false><<<grid, 256, 0, st>>>(X, q, n, bc, p, ng, v, nt, strip, nsx, rowpart, colpart);
  KQR_LAUNCH_CHECK();
  packed_reduce(rowpart, colpart, n, strip, u, ldu, st);
  KQR_CHECK_HIP(hipFreeAsync(buf, st));
}

template <int KP>
static void kapply_otf_mfma_p(const float* Xr, const float* qr, int64_t nr, const float* Xc, const float* qc,
                              int64_t nc, int p, KernelSpec ks, const double* v, double* u, int64_t ldu, double scale,
                              double shift, bool exact, hipStream_t st, double* scratch, size_t scratch_doubles) {
  if (Xr == Xc && qr == qc && nr == nc && scale == 1.0 && shift == 0.0 && otf_sym_fits(nr)) {  // square: symmetric
    kapply_otf_mfma_sym<KP>(Xr, qr, nr, p, ks, v, u, ldu, exact, st, scratch, scratch_doubles);
    return;
  }
  const int64_t rblk = (nr + 127) / 128;
  int64_t nslice = otf_slices(rblk, nc);
  nslice = std::min<int64_t>(nslice, 65535);
  int64_t per = (nc + nslice - 1) / nslice;
  const int64_t stage = KP > 16 ? kB3Cols : kMfmaCols;
  per = (per + stage - 1) / stage * stage;
  nslice = (nc + per - 1) / per;
  const size_t part_bytes = (size_t(nslice) * size_t(nr) * sizeof(double) + 255) / 256 * 256;
  const size_t split_bytes = KP > 16 ? size_t(nc) * kB3Stride * sizeof(uint16_t) : 0;
  char* buf = nullptr;
  KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&buf), part_bytes + split_bytes, st));
  double* part = reinterpret_cast<double*>(buf);
  const dim3 grid((unsigned)rblk, (unsigned)nslice);
  const float ng = -float(ks.gamma) * kLog2e;
  if (KP > 16) {  // BF16x3 Gram: 6 MFMAs of K = 32 against KP/4 FP32 ones
    uint16_t* bc = reinterpret_cast<uint16_t*>(buf + part_bytes);
    const bool aug = p <= 30;
    const dim3 sgrid((unsigned)((nc * 4 + 255) / 256));
    if (aug) kotf_split_cols_kernel<true><<<sgrid, 256, 0, st>>>(Xc, qc, nc, p, ng, bc);
    else kotf_split_cols_kernel<false><<<sgrid, 256, 0, st>>>(Xc, qc, nc, p, ng, bc);
    KQR_LAUNCH_CHECK();
    if (aug && exact) kapply_otf_mfma3_kernel<true, true><<<grid, 256, 0, st>>>(Xr, qr, nr, bc, qc, nc, p, ng, v, per, part);
    else if (aug) kapply_otf_mfma3_kernel<false, true><<<grid, 256, 0, st>>>(Xr, qr, nr, bc, qc, nc, p, ng, v, per, part);
    else if (exact) kapply_otf_mfma3_kernel<true, false><<<grid, 256, 0, st>>>(Xr, qr, nr, bc, qc, nc, p, ng, v, per, part);
    else kapply_otf_mfma3_kernel<false, false><<<grid, 256, 0, st>>>(Xr, qr, nr, bc, qc, nc, p, ng, v, per, part);
  } else if (exact) {
    kapply_otf_mfma_kernel<KP, true><<<grid, 256, 0, st>>>(Xr, qr, nr, Xc, qc, nc, p, ng, v, per, part);
  } else {
    kapply_otf_mfma_kernel<KP, false><<<grid, 256, 0, st>>>(Xr, qr, nr, Xc, qc, nc, p, ng, v, per, part);
  }
  KQR_LAUNCH_CHECK();
  otf_reduce_kernel<<<dim3((unsigned)((nr + 255) / 256)), 256, 0, st>>>(part, int(nslice), nr, u, ldu, scale, shift);
  KQR_LAUNCH_CHECK();
  KQR_CHECK_HIP(hipFreeAsync(buf, st));
}

void kapply_otf(const float* Xr, const float* sqr, int64_t nr, const float* Xc, const float* sqc,
                int64_t nc, int p, KernelSpec ks, const double* v64, double* u, int64_t ldu,
                double out_scale, double out_shift, hipStream_t st, bool exact, double* scratch,
                size_t scratch_doubles) {
  if (nr <= 0) return;
  if (ks.kind == KQR_RBF && p <= 32) {
#define KQR_OTF_MFMA(KP) \
  kapply_otf_mfma_p<KP>(Xr, sqr, nr, Xc, sqc, nc, p, ks, v64, u, ldu, out_scale, out_shift, exact, st, scratch, \
                        scratch_doubles)
    switch ((p + 3) / 4) {
      case 1:
      case 2: KQR_OTF_MFMA(8); return;
      case 3: KQR_OTF_MFMA(12); return;
      case 4: KQR_OTF_MFMA(16); return;
      case 5: KQR_OTF_MFMA(20); return;
      case 6: KQR_OTF_MFMA(24); return;
      case 7: KQR_OTF_MFMA(28); return;
      default: KQR_OTF_MFMA(32); return;
    }
#undef KQR_OTF_MFMA
  }
  KQR_DISPATCH_P(p, kapply_otf_p, Xr, sqr, nr, Xc, sqc, nc, p, ks, v64, u, ldu, out_scale, out_shift, exact, st);
}

// ================================================================= K build on the matrix cores
// RBF with p <= 32: the Gram term of every 16 x 16 block on the matrix cores
// (v_mfma_f32_16x16x32_bf16) from the exact BF16x3 split of both sides (as
// the on-the-fly applies), with the norms and the exponent's scale folded into
// the spare coordinates when p <= 30 (the matrix cores then return
// c d_ij, c = -gamma log2(e)), so an entry costs the lanes a clamp, the
// exponential, the diagonal test and its share of a store.  Both sides are
// split once per build into buffers of 96 halves per point (row side
// [x, 1, q], column side [-2 c x, c q, c]; without the fold [x] and [-2 x]).
// FP32 storage takes all six significant products.  BF16 storage takes the
// three leading ones (hi.hi, hi.mid, mid.hi): the dropped ones are at most
// 3 2^-16 sum_k |a_k| |b_k|, and that sum is at most 2 |c| (q_i + q_j)
// (2 |x_i . x_j| <= q_i + q_j), so the entry moves by a relative
// 3 2^-15 gamma (q_i + q_j) at most.  The three products are used only when
// gamma max_i q_i <= 16 / 3, which keeps that below 2^-10, a quarter of
// BF16's unit roundoff 2^-8; inputs far from the origin get the six.
//
// Operand roles: the A operand carries 16 columns j of K and the B operand
// 16 rows i, so the lane that receives C[4 g + r][l] holds K[i0 + l][j0 +
// 4 g + r], r = 0..3.  A workgroup is four waves of 32 rows each (two 16-row
// strips as B operands held in registers); a step covers 64 columns (four
// 16-column blocks, whose column parts each wave loads once from L2, 192
// bytes per column, and uses for both strips).  The step's 32 x 64 entries of
// a wave go through its own LDS slab and leave as whole rows: 16-byte stores,
// 256 contiguous bytes per row (FP32) or 128 (BF16), so every store writes
// full 128-byte lines (the MFMA layout alone would give 64- or 32-byte pieces
// per row and instruction).
//   full layout  : 128 rows x `cols` columns of the n x ldk matrix per workgroup
//                  (columns n..ldk-1 written as 0, rows >= n not written;
//                  ldk and `cols` multiples of 64);
//   packed layout: one 128 x 128 upper-triangle tile per workgroup (entries
//                  beyond n written as 0, as the tile layout requires).
// K_ii is set to exactly 1 (d_ii := 0).
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

constexpr int kBuildStep = 64;               // columns per step
constexpr int kBuildSlab = kBuildStep + 4;   // LDS row of a wave's slab (floats), padded against bank conflicts

template <bool AUG, bool BF, bool PACKED>
__global__ __launch_bounds__(256) void kbuild_b3_kernel(const uint16_t* __restrict__ Pr, const uint16_t* __restrict__ Sc,
                                                        const float* __restrict__ q, int64_t n, float ng,
                                                        void* __restrict__ Kout, int64_t ldk, int64_t nt,
                                                        int64_t cols, const float* __restrict__ qmax, float qlim) {
  // a wave's slab: 32 rows x 64 entries, FP32 or (BF16 storage) the rounded BF16 values
  __shared__ __align__(16) float slab[4][32][kBuildSlab];
  typedef uint16_t bslab_row[2 * kBuildSlab];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: block tests branch on scalars
  const int li = lane & 15, lg = lane >> 4;
  int64_t rbase, cbeg, cend;
  size_t tile_base = 0;
  if (PACKED) {
    const int64_t t = blockIdx.x;
    int64_t lo = 0, hi = nt - 1;  // largest I whose first tile index is <= t
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (pk_tile_index(mid, mid, nt) <= t) lo = mid;
      else hi = mid - 1;
    }
    const int64_t J = lo + (t - pk_tile_index(lo, lo, nt));
    rbase = lo * kPkT;
    cbeg = J * kPkT;
    cend = cbeg + kPkT;
    tile_base = size_t(t) * kPkT * kPkT;
  } else {
    rbase = int64_t(blockIdx.x) * 128;
    cbeg = int64_t(blockIdx.y) * cols;
    cend = min(ldk, cbeg + cols);
  }
  const int64_t wrow = rbase + 32 * wave;  // this wave's first row
  // B operands: rows wrow + 16 s + li, coordinates 8 lg .. 8 lg + 7
  bf16x8_t bh[2], bm[2], bl[2];
  float qi[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int64_t ic = min(wrow + 16 * s + li, n - 1);  // rows past n: any valid point (entries not kept)
    bh[s] = *reinterpret_cast<const bf16x8_t*>(Pr + ic * kB3Stride + 8 * lg);
    bm[s] = *reinterpret_cast<const bf16x8_t*>(Pr + ic * kB3Stride + 32 + 8 * lg);
    bl[s] = *reinterpret_cast<const bf16x8_t*>(Pr + ic * kB3Stride + 64 + 8 * lg);
    qi[s] = AUG ? 0.f : q[ic];
  }
  const uint32_t col_off = uint32_t(li) * kB3Stride + 8 * lg;  // this lane's column part within a block
  float (*sl)[kBuildSlab] = slab[wave];
  bslab_row* bsl = reinterpret_cast<bslab_row*>(slab[wave]);  // BF16 view: rows of 2 kBuildSlab halves
  // BF16 storage: three products when the largest squared norm allows (see
  // above); one instantiation of the step loop per case, chosen once
  auto steps = [&](auto three_c) {
    constexpr bool three = decltype(three_c)::value;
    for (int64_t jb = cbeg; jb < cend; jb += kBuildStep) {
      // the column parts of the whole step are requested at once: one L2 round
      // trip per step instead of one per 16-column block
      bf16x8_t ahs[kBuildStep / 16], ams[kBuildStep / 16], als[kBuildStep / 16];
      if (jb + kBuildStep <= n) {  // (uniform) whole step inside: a scalar base per block, the lane's offset fixed
#pragma unroll
        for (int blk = 0; blk < kBuildStep / 16; ++blk) {
          const uint16_t* cb = Sc + (jb + 16 * blk) * kB3Stride;
          ahs[blk] = *reinterpret_cast<const bf16x8_t*>(cb + col_off);
          ams[blk] = *reinterpret_cast<const bf16x8_t*>(cb + col_off + 32);
          if constexpr (!three) als[blk] = *reinterpret_cast<const bf16x8_t*>(cb + col_off + 64);
        }
      } else {
#pragma unroll
        for (int blk = 0; blk < kBuildStep / 16; ++blk) {
          const int64_t jc = min(jb + 16 * blk + li, n - 1);  // columns past n: any valid point (written as 0)
          ahs[blk] = *reinterpret_cast<const bf16x8_t*>(Sc + jc * kB3Stride + 8 * lg);
          ams[blk] = *reinterpret_cast<const bf16x8_t*>(Sc + jc * kB3Stride + 32 + 8 * lg);
          if constexpr (!three) als[blk] = *reinterpret_cast<const bf16x8_t*>(Sc + jc * kB3Stride + 64 + 8 * lg);
        }
      }
      // Gram blocks: the two strips' product chains interleaved, and the next
      // block's MFMAs issued before this block's exponentials
      auto gram = [&](int blk, f32x4_t* c) {
        const bf16x8_t ah = ahs[blk], am = ams[blk];
        c[0] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        c[1] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        if constexpr (three) {
          c[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[0], c[0], 0, 0, 0);
          c[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[1], c[1], 0, 0, 0);
          c[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm[0], c[0], 0, 0, 0);
          c[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm[1], c[1], 0, 0, 0);
          c[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[0], c[0], 0, 0, 0);
          c[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[1], c[1], 0, 0, 0);
          return;
        }
        // smallest products first
        const bf16x8_t al = als[blk];
        c[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm[0], c[0], 0, 0, 0);
        c[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm[1], c[1], 0, 0, 0);
        c[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[0], c[0], 0, 0, 0);
        c[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[1], c[1], 0, 0, 0);
        c[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[0], c[0], 0, 0, 0);
        c[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[1], c[1], 0, 0, 0);
        c[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[0], c[0], 0, 0, 0);
        c[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[1], c[1], 0, 0, 0);
        c[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm[0], c[0], 0, 0, 0);
        c[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm[1], c[1], 0, 0, 0);
        c[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[0], c[0], 0, 0, 0);
        c[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[1], c[1], 0, 0, 0);
      };
      f32x4_t cur[2], nxt[2];
      gram(0, cur);
#pragma unroll
      for (int blk = 0; blk < kBuildStep / 16; ++blk) {
        if (blk + 1 < kBuildStep / 16) gram(blk + 1, nxt);
        const int64_t j0 = jb + 16 * blk + 4 * lg;  // this lane's four columns j0 .. j0 + 3
        float qj[4] = {0.f, 0.f, 0.f, 0.f};
        if (!AUG) {
#pragma unroll
          for (int r = 0; r < 4; ++r) qj[r] = q[min(j0 + r, n - 1)];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const f32x4_t c = cur[s];
          const int64_t iblk = wrow + 16 * s, jblk = jb + 16 * blk;
          f32x4_t e;
          // ng < 0 and d >= 0, so the entry is exp2(min(ng d, 0)) = min(exp2(ng d), 1): the
          // clamp to [0, 1] rides on the exponential as its output modifier
#pragma unroll
          for (int r = 0; r < 4; ++r)
            e[r] = __builtin_amdgcn_fmed3f(kexp2(AUG ? c[r] : ng * (qi[s] + qj[r] + c[r])), 0.f, 1.f);
          if (iblk == jblk || iblk + 16 > n || jblk + 16 > n) {  // (uniform) diagonal or ragged block
            // 32-bit tests against the block's valid extents (both blocks start on multiples of 16)
            const int64_t ri = n - iblk, rj = n - jblk;
            const int ni = ri < 16 ? int(ri) : 16, nj = rj < 16 ? int(rj) : 16;
            const bool diag = iblk == jblk;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int jl = 4 * lg + r;
              e[r] = (jl < nj && li < ni) ? ((diag && jl == li) ? 1.f : e[r]) : 0.f;
            }
          }
          if (BF) {  // round to BF16 here: half the LDS traffic
            u32x2_t w;
            w[0] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{e[0], e[1]}, bf16x2_t));
            w[1] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{e[2], e[3]}, bf16x2_t));
            *reinterpret_cast<u32x2_t*>(&bsl[16 * s + li][16 * blk + 4 * lg]) = w;
          } else {
            *reinterpret_cast<f32x4_t*>(&sl[16 * s + li][16 * blk + 4 * lg]) = e;
          }
        }
        cur[0] = nxt[0];
        cur[1] = nxt[1];
      }
      __syncthreads();  // the slab is complete (each wave reads only its own)
      if (BF) {
        // a row is 64 BF16 = 128 bytes = 8 lanes x 16 bytes; eight rows per store
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int rr = 8 * k + (lane >> 3), cc = 8 * (lane & 7);
          const u32x4_t w = *reinterpret_cast<const u32x4_t*>(&bsl[rr][cc]);
          const int64_t i = wrow + rr;
          if (PACKED) {
            const size_t off = tile_base + size_t(i - rbase) * kPkT + size_t(jb - cbeg + cc);
            __builtin_nontemporal_store(w, reinterpret_cast<u32x4_t*>(static_cast<uint16_t*>(Kout) + off));
          } else if (i < n) {
            const size_t off = size_t(i) * size_t(ldk) + size_t(jb + cc);
            __builtin_nontemporal_store(w, reinterpret_cast<u32x4_t*>(static_cast<uint16_t*>(Kout) + off));
          }
        }
      } else {
        // a row is 64 FP32 = 256 bytes = 16 lanes x 16 bytes; four rows per store
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int rr = 4 * k + (lane >> 4), cc = 4 * (lane & 15);
          const f32x4_t x = *reinterpret_cast<const f32x4_t*>(&sl[rr][cc]);
          const int64_t i = wrow + rr;
          if (PACKED) {
            const size_t off = tile_base + size_t(i - rbase) * kPkT + size_t(jb - cbeg + cc);
            __builtin_nontemporal_store(x, reinterpret_cast<f32x4_t*>(static_cast<float*>(Kout) + off));
          } else if (i < n) {
            const size_t off = size_t(i) * size_t(ldk) + size_t(jb + cc);
            __builtin_nontemporal_store(x, reinterpret_cast<f32x4_t*>(static_cast<float*>(Kout) + off));
          }
        }
      }
      __syncthreads();  // the slab is free for the next step
    }
  };
  if (BF && *qmax <= qlim) steps(std::true_type{});
  else steps(std::false_type{});
}

// Columns per workgroup of the full-layout build.
constexpr int64_t kBuildCols = 1024;

// out[0] = max_i q_i (one workgroup of 1024 threads)
__global__ __launch_bounds__(1024) void qmax_kernel(const float* __restrict__ q, int64_t n, float* __restrict__ out) {
  __shared__ float sh[16];
  float m = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, q[i]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) m = fmaxf(m, sh[w]);
    out[0] = fmaxf(m, sh[0]);
  }
}

bool kbuild_mfma(const float* X, const float* q, int64_t n, int p, KernelSpec ks, int dtype, void* K, int64_t ldk,
                 int layout, hipStream_t st) {
  if (ks.kind != KQR_RBF || p > 32 || n <= 0) return false;
  if (layout == 0 && ldk % kBuildStep != 0) return false;  // the stores cover 64-column steps up to ldk
  const bool aug = p <= 30, bf = dtype == KQR_BF16;
  const float ng = -float(ks.gamma) * kLog2e;
  uint16_t* buf = nullptr;
  const size_t half_bytes = size_t(n) * kB3Stride * sizeof(uint16_t);
  KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&buf), 2 * half_bytes + 256, st));
  uint16_t* Pr = buf;                      // row side
  uint16_t* Sc = buf + size_t(n) * kB3Stride;  // column side (scaled)
  float* qmax = reinterpret_cast<float*>(buf + 2 * size_t(n) * kB3Stride);
  const float qlim = float(16.0 / (3.0 * ks.gamma));  // three products when max q <= qlim
  if (bf) {
    qmax_kernel<<<1, 1024, 0, st>>>(q, n, qmax);
    KQR_LAUNCH_CHECK();
  }
  const dim3 sgrid((unsigned)((n * 4 + 255) / 256));
  if (aug) {
    kotf_split_cols_kernel<true, false><<<sgrid, 256, 0, st>>>(X, q, n, p, ng, Pr);
    kotf_split_cols_kernel<true, true><<<sgrid, 256, 0, st>>>(X, q, n, p, ng, Sc);
  } else {
    kotf_split_cols_kernel<false, false><<<sgrid, 256, 0, st>>>(X, q, n, p, ng, Pr);
    kotf_split_cols_kernel<false, true><<<sgrid, 256, 0, st>>>(X, q, n, p, ng, Sc);
  }
  KQR_LAUNCH_CHECK();
  const int64_t nt = (n + kPkT - 1) / kPkT;
  dim3 grid;
  if (layout == 1) grid = dim3((unsigned)packed_tile_count(n));
  else grid = dim3((unsigned)((n + 127) / 128), (unsigned)((ldk + kBuildCols - 1) / kBuildCols));
#define KQR_B3(A, B, P) \
  kbuild_b3_kernel<A, B, P><<<grid, 256, 0, st>>>(Pr, Sc, q, n, ng, K, ldk, nt, kBuildCols, qmax, qlim)
  if (layout == 1) {
    if (aug && bf) KQR_B3(true, true, true);
    else if (aug) KQR_B3(true, false, true);
    else if (bf) KQR_B3(false, true, true);
    else KQR_B3(false, false, true);
  } else {
    if (aug && bf) KQR_B3(true, true, false);
    else if (aug) KQR_B3(true, false, false);
    else if (bf) KQR_B3(false, true, false);
    else KQR_B3(false, false, false);
  }
#undef KQR_B3
  KQR_LAUNCH_CHECK();
  KQR_CHECK_HIP(hipFreeAsync(buf, st));
  return true;
}

// ================================================================= one kernel row
template <bool BF16>
__global__ void krow_from_mat_kernel(const void* __restrict__ K, int64_t ldk, int64_t n, int64_t s,
                                     double* __restrict__ out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (BF16) out[j] = bf16_to_f32(static_cast<const uint16_t*>(K)[s * ldk + j]);
  else out[j] = static_cast<const float*>(K)[s * ldk + j];
}

template <int PMAX, bool LAP>
__global__ void krow_from_x_kernel(const float* __restrict__ X, const float* __restrict__ q,
                                   int64_t n, int p, float ng, int64_t s, double* __restrict__ out) {
  __shared__ float xs[PMAX];
  if (threadIdx.x < PMAX) xs[threadIdx.x] = threadIdx.x < p ? X[s * p + threadIdx.x] : 0.f;
  __syncthreads();
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  float xj[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) xj[k] = k < p ? X[j * p + k] : 0.f;
  float d = pair_dist<PMAX, LAP>(xs, LAP ? 0.f : q[s], xj, LAP ? 0.f : q[j]);
  if (j == s) d = 0.f;
  out[j] = kexp2(ng * d);
}

template <int PMAX>
static void krow_p(const float* X, const float* q, int64_t n, int p, KernelSpec ks, int64_t s,
                   double* out, hipStream_t st) {
  const dim3 grid((unsigned)((n + 255) / 256));
  const float ng = -float(ks.gamma) * kLog2e;
  if (ks.kind == KQR_LAPLACIAN) krow_from_x_kernel<PMAX, true><<<grid, 256, 0, st>>>(X, q, n, p, ng, s, out);
  else krow_from_x_kernel<PMAX, false><<<grid, 256, 0, st>>>(X, q, n, p, ng, s, out);
  KQR_LAUNCH_CHECK();
}

void kernel_row(const KMat& km, const float* X, const float* sqn, int64_t n, int p, KernelSpec ks,
                int64_t s, double* out, hipStream_t st) {
  if (km.K && km.layout == 1) {
    kernel_row_packed(km, n, s, out, st);
    return;
  }
  if (km.K) {
    const dim3 grid((unsigned)((n + 255) / 256));
    if (km.dtype == KQR_BF16) krow_from_mat_kernel<true><<<grid, 256, 0, st>>>(km.K, km.ld, n, s, out);
    else krow_from_mat_kernel<false><<<grid, 256, 0, st>>>(km.K, km.ld, n, s, out);
    KQR_LAUNCH_CHECK();
    return;
  }
  KQR_DISPATCH_P(p, krow_p, X, sqn, n, p, ks, s, out, st);
}

// ================================================================= skinny mat-vec
// 16 lanes per row (4 rows per wave at a time, 4 such row slots per wave):
// a lane reads 16-byte pieces of its row 64 columns apart, x sits in LDS, and
// a 4-step shuffle reduction inside each 16-lane group finishes 4 rows at once.
// (Workgroup blk of the launch; the body also serves the batched PCG steps.)
__device__ __forceinline__ void gemv_skinny_body(const float* __restrict__ A, int64_t lda, int64_t nrows, int ncols,
                                                 const double* __restrict__ x, double* __restrict__ y, int blk) {
  __shared__ double xs[1024 + 4];
  for (int k = threadIdx.x; k < ncols; k += 256) xs[k] = x[k];
  for (int k = ncols + threadIdx.x; k < ((ncols + 3) & ~3); k += 256) xs[k] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, t = lane & 15;
  const int64_t wrow0 = (int64_t(blk) * 4 + wave) * 16;
  const int nvec = ncols >> 2;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const float* rows[4];
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    const int64_t r = min(wrow0 + sl * 4 + g, nrows - 1);
    rows[sl] = A + r * lda;
  }
  for (int c = t; c < nvec; c += 16) {
    float4 v[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) v[sl] = reinterpret_cast<const float4*>(rows[sl])[c];
    const double x0 = xs[4 * c], x1 = xs[4 * c + 1], x2 = xs[4 * c + 2], x3 = xs[4 * c + 3];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      acc[sl] = fma(double(v[sl].x), x0, acc[sl]);
      acc[sl] = fma(double(v[sl].y), x1, acc[sl]);
      acc[sl] = fma(double(v[sl].z), x2, acc[sl]);
      acc[sl] = fma(double(v[sl].w), x3, acc[sl]);
    }
  }
  for (int c = nvec * 4 + t; c < ncols; c += 16) {
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) acc[sl] = fma(double(rows[sl][c]), xs[c], acc[sl]);
  }
#pragma unroll
  for (int sl = 0; sl < 4; ++sl)
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) acc[sl] += __shfl_xor(acc[sl], off, 16);
  if (t == 0) {
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      const int64_t r = wrow0 + sl * 4 + g;
      if (r < nrows) y[r] = acc[sl];
    }
  }
}

__global__ __launch_bounds__(256) void gemv_skinny_kernel(const float* __restrict__ A, int64_t lda, int64_t nrows,
                                                          int ncols, const double* __restrict__ x,
                                                          double* __restrict__ y) {
  gemv_skinny_body(A, lda, nrows, ncols, x, y, int(blockIdx.x));
}

// Batched PCG steps: Fs = F s_{1..rank} of every fit with rank > 0, each
// over its range of workgroups (64 rows each).
__global__ __launch_bounds__(256) void wood_fs_steps_kernel(const PcgStepDesc* __restrict__ d,
                                                            const int* __restrict__ first, int nf) {
  const int f = step_of_block(first, nf, int(blockIdx.x));
  const PcgStepDesc& e = d[f];
  gemv_skinny_body(e.F, e.ldf, e.n, e.rank, e.s, e.Fs, int(blockIdx.x) - first[f]);
}

void launch_wood_fs_steps(const PcgStepDesc* d, const int* fs_first, int nf, int total, hipStream_t st) {
  if (nf <= 0 || total <= 0) return;
  wood_fs_steps_kernel<<<total, 256, 0, st>>>(d, fs_first, nf);
  KQR_LAUNCH_CHECK();
}

int pcg_step_fs_blocks(const PcgStepDesc& d) { return d.rank > 0 ? int((d.n + 63) / 64) : 0; }

void gemv_skinny(const float* A, int64_t lda, int64_t nrows, int64_t ncols, const double* x, double* y,
                 hipStream_t st) {
  if (nrows <= 0) return;
  if (ncols > 1024 || (lda & 3)) fail(KQR_EINVAL, "gemv_skinny: ncols <= 1024 and lda % 4 == 0 required");
  gemv_skinny_kernel<<<dim3((unsigned)((nrows + 63) / 64)), 256, 0, st>>>(A, lda, nrows, int(ncols), x, y);
  KQR_LAUNCH_CHECK();
}

// ================================================================= FP64 -> FP32
__global__ void to_f32_kernel(const double* __restrict__ src, int64_t n, int m, int64_t lds,
                              float* __restrict__ dst, int64_t ldd) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * m) return;
  const int64_t i = t / m;
  const int k = int(t % m);
  dst[i * ldd + k] = float(src[i * lds + k]);
}

void to_f32(const double* src, int64_t n, int m, int64_t lds, float* dst, int64_t ldd, hipStream_t st) {
  if (n <= 0) return;
  const int64_t tot = n * m;
  to_f32_kernel<<<dim3((unsigned)((tot + 255) / 256)), 256, 0, st>>>(src, n, m, lds, dst, ldd);
  KQR_LAUNCH_CHECK();
}

}  // namespace kqr
