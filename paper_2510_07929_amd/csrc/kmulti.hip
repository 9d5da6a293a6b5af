// Batched kernel operators:
//  * K V for up to 16 right-hand sides on the matrix cores (one pass over K
//    serves every column: the tau-batch of kqr_fit_multi_tau);
//  * K_i v_i for many independent problems of different sizes in one launch
//    (the uneven batch of kqr_fit_batch): workgroups are dealt out over the
//    (problem, row block) pairs of all problems.
#include "kqr_internal.h"
#include "kmulti.h"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace kqr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kKC = 256;       // columns of K per LDS stage of V
constexpr int kVpad = kKC + 8; // padded LDS row (bank spread)
}  // namespace

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// U[seg] rows = K[rows, cols of segment] V[cols, 0:16].  Block = 4 waves, each
// wave a 16-row strip.  V (row-major, 16 FP32 columns, rows padded with zeros
// up to ld_rows) is staged transposed in LDS per kKC columns.  The MFMA
// accumulators (FP32, two independent chains) are flushed into FP64 after
// every stage.  K is streamed with 16-byte non-temporal loads, 64 contiguous
// bytes per row per load instruction (the four lanes of a row are adjacent),
// and (PF) the next step's loads are issued before the current step's MFMAs.
// A lane issues NLD (4 or 8) loads per step, NLD KB in flight per wave.
//  FP32 K: v_mfma_f32_16x16x4f32; a step is 16 NLD columns, a lane holds
//          4 NLD entries of its row (columns 16q + 4g + e for lane group g).
//  BF16 K: v_mfma_f32_16x16x32_bf16 with V split into hi + lo BF16 parts; a
//          step is 32 NLD columns, a lane holds 8 NLD entries (32q + 8g + e).
// Only the last step of a segment can be partial; it is read element-wise with
// zero fill, so nothing beyond column ncols is touched.
template <bool BF16, int NLD, bool PF>
__global__ __launch_bounds__(256) void kv_mfma_kernel(const void* __restrict__ K, int64_t ldk, int64_t n,
                                                      int64_t ncols, const float* __restrict__ V,
                                                      int64_t seg_cols, double* __restrict__ out) {
  constexpr int STEP = (BF16 ? 32 : 16) * NLD;
  __shared__ float vs[BF16 ? 1 : 16][BF16 ? 1 : kVpad];
  __shared__ uint16_t vh[BF16 ? 16 : 1][BF16 ? kVpad : 1];
  __shared__ uint16_t vl[BF16 ? 16 : 1][BF16 ? kVpad : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t row0 = int64_t(blockIdx.x) * 64 + wave * 16;
  const int64_t my_row = min(row0 + li, n - 1);
  const int64_t c0 = int64_t(blockIdx.y) * seg_cols;
  const int64_t c1 = min(ncols, c0 + seg_cols);
  double acc64[4] = {0.0, 0.0, 0.0, 0.0};
  const char* krow = static_cast<const char*>(K) + my_row * ldk * (BF16 ? 2 : 4);
  // a[q] = 16 bytes of the row at column col + (BF16 ? 32 : 16) q + (BF16 ? 8 : 4) g
  auto load_step = [&](int64_t col, u32x4 (&a)[NLD]) {
    const int per = BF16 ? 8 : 4;  // entries per 16 bytes
    if (col + STEP <= c1) {
#pragma unroll
      for (int q = 0; q < NLD; ++q)
        a[q] = __builtin_nontemporal_load(
            reinterpret_cast<const u32x4*>(krow + (col + q * 4 * per + lg * per) * (BF16 ? 2 : 4)));
    } else {
#pragma unroll
      for (int q = 0; q < NLD; ++q) {
        const int64_t cc = col + q * 4 * per + lg * per;
        if (BF16) {
          const uint16_t* kr = reinterpret_cast<const uint16_t*>(krow);
          uint32_t w[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t lo = (cc + 2 * e < c1) ? kr[cc + 2 * e] : 0u;
            const uint32_t hi = (cc + 2 * e + 1 < c1) ? kr[cc + 2 * e + 1] : 0u;
            w[e] = lo | (hi << 16);
          }
          a[q] = u32x4{w[0], w[1], w[2], w[3]};
        } else {
          const float* kr = reinterpret_cast<const float*>(krow);
          uint32_t w[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) w[e] = (cc + e < c1) ? __float_as_uint(kr[cc + e]) : 0u;
          a[q] = u32x4{w[0], w[1], w[2], w[3]};
        }
      }
    }
  };
  for (int64_t cb = c0; cb < c1; cb += kKC) {
    const int cnt = int(min<int64_t>(kKC, c1 - cb));
    u32x4 a[NLD], an[NLD];
    load_step(cb, a);  // independent of V: in flight while V is staged
    __syncthreads();
    for (int e = threadIdx.x; e < kKC * 16; e += 256) {
      const int kk = e >> 4, j = e & 15;
      const float val = kk < cnt ? V[(cb + kk) * 16 + j] : 0.f;
      if (BF16) {
        const uint16_t h = f2bf(val);
        vh[j][kk] = h;
        vl[j][kk] = f2bf(val - __uint_as_float(uint32_t(h) << 16));
      } else {
        vs[j][kk] = val;
      }
    }
    __syncthreads();
    f32x4 accA = {0.f, 0.f, 0.f, 0.f}, accB = {0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < cnt; kk += STEP) {
      const bool more = kk + STEP < cnt;
      if (PF && more) load_step(cb + kk + STEP, an);
      if (BF16) {
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
          const bf16x8 av = __builtin_bit_cast(bf16x8, a[q]);
          const int off = kk + 32 * q + 8 * lg;
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&vh[li][off]);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&vl[li][off]);
          accA = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bh, accA, 0, 0, 0);
          accB = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl, accB, 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
          const f32x4 b = *reinterpret_cast<const f32x4*>(&vs[li][kk + 16 * q + 4 * lg]);
          const f32x4 av = __builtin_bit_cast(f32x4, a[q]);
          accA = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0], b[0], accA, 0, 0, 0);
          accB = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1], b[1], accB, 0, 0, 0);
          accA = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2], b[2], accA, 0, 0, 0);
          accB = __builtin_amdgcn_mfma_f32_16x16x4f32(av[3], b[3], accB, 0, 0, 0);
        }
      }
      if (more) {
        if (PF) {
#pragma unroll
          for (int q = 0; q < NLD; ++q) a[q] = an[q];
        } else {
          load_step(cb + kk + STEP, a);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[r] += double(accA[r]) + double(accB[r]);
  }
  // accumulator layout of a 16x16 MFMA: lane holds rows 4*(lane/16)+r, column lane%16
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + 4 * lg + r;
    if (row < n) out[(int64_t(blockIdx.y) * n + row) * 16 + li] = acc64[r];
  }
}

// Row-streamed K V: the block owns 64 rows; per stage it reads a 64-row tile
// of K (FP32: 128 columns, BF16: 256 columns; 32 KB) with 16-byte
// non-temporal loads, 512 contiguous bytes per row and load instruction (the
// access pattern of the single-vector K-apply), writes it to LDS, and each
// wave forms its 16-row strip on the matrix cores from LDS.  The next stage's
// tile is loaded into registers while the current one is multiplied.  Lane
// group g of a strip takes the columns [g C/4, (g+1) C/4) of the stage, so
// every lane reads contiguous 16-byte pieces of K and V from LDS.
// With MX = 1, 2 or 4 (FP32 K only) the same staged tile also serves that many
// exact columns: thread t forms, for rows 4 (t/16) .. +3 of the tile and the
// columns [8 (t%16), 8 (t%16) + 8) of the stage, FP64 products of the FP32
// entries with FP64 Vx (n x 4) and FP64 sums (the exact operator), so exact
// applies cost no extra pass over K.  The FP64 work and its registers grow
// with MX: with one column the kernel keeps three waves per SIMD (as without
// exact columns), with two or four it runs two.
template <bool BF16, int MX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MX == 1 ? 3 : 1))) void kv_staged_kernel(const void* __restrict__ K, int64_t ldk, int64_t n,
                                                        int64_t ncols, const float* __restrict__ V,
                                                        const uint16_t* __restrict__ Vhl, int64_t seg_cols,
                                                        double* __restrict__ out, const double* __restrict__ Vx,
                                                        double* __restrict__ outx) {
  static_assert(MX == 0 || ((MX == 1 || MX == 2 || MX == kKvMaxExact) && !BF16),
                "exact columns (1, 2 or 4) ride on FP32 stages only");
  constexpr int COLS = BF16 ? 256 : 128;   // columns per stage
  constexpr int PER = BF16 ? 8 : 4;        // entries per 16 bytes
  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int KPAD = COLS + (BF16 ? 8 : 4);  // LDS row length in entries (row start bank = 4 i mod 64)
  constexpr int QCOL = COLS / 4;               // columns per lane group
  __shared__ __attribute__((aligned(16))) unsigned char ks[64 * KPAD * ESZ];
  __shared__ __attribute__((aligned(16))) float vs[BF16 ? 1 : 16][BF16 ? 4 : COLS + 4];
  __shared__ __attribute__((aligned(16))) uint16_t vh[BF16 ? 16 : 1][BF16 ? COLS + 8 : 8];
  __shared__ __attribute__((aligned(16))) uint16_t vl[BF16 ? 16 : 1][BF16 ? COLS + 8 : 8];
  // exact columns transposed, 8 columns per 16-lane slice padded to 10 (the
  // 16 lanes' 16-byte reads then start on distinct banks)
  __shared__ __attribute__((aligned(16))) double vxs[MX > 0 ? kKvMaxExact : 1][MX > 0 ? 16 * 10 : 2];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t row_base = int64_t(blockIdx.x) * 64;
  const int64_t c0 = int64_t(blockIdx.y) * seg_cols;
  const int64_t c1 = min(ncols, c0 + seg_cols);
  const char* Kb = static_cast<const char*>(K);
  const int tr = t >> 5, tc = t & 31;  // loader: row offset in a group of 8 rows, 16-byte chunk in the row
  auto load_stage = [&](int64_t cb, u32x4 (&r)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t row = min(row_base + q * 8 + tr, n - 1);
      const int64_t cc = cb + tc * PER;
      const char* src = Kb + (row * ldk + cc) * ESZ;
      if (cc + PER <= c1) {
        r[q] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src));
      } else {
        uint32_t w[4];
        if (BF16) {
          const uint16_t* kr = reinterpret_cast<const uint16_t*>(Kb) + row * ldk;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t lo = (cc + 2 * e < c1) ? kr[cc + 2 * e] : 0u;
            const uint32_t hi = (cc + 2 * e + 1 < c1) ? kr[cc + 2 * e + 1] : 0u;
            w[e] = lo | (hi << 16);
          }
        } else {
          const float* kr = reinterpret_cast<const float*>(Kb) + row * ldk;
#pragma unroll
          for (int e = 0; e < 4; ++e) w[e] = (cc + e < c1) ? __float_as_uint(kr[cc + e]) : 0u;
        }
        r[q] = u32x4{w[0], w[1], w[2], w[3]};
      }
    }
  };
  // The stage's rows of V (and of the exact columns' Vx) in 16-byte pieces at
  // clamped rows, loaded one stage ahead with K; rows past the segment are
  // zeroed when written to LDS.  FP32: thread t takes half h = t & 1 of row
  // t / 2 (8 floats); BF16: all 64 bytes of row t (16 hi + 16 lo halves);
  // exact: threads t < 128 take the 4 doubles of row t.
  constexpr int NV = BF16 ? 4 : 2;
  auto load_v = [&](int64_t cb, u32x4 (&pv)[NV], u32x4 (&px)[2]) {
    const int cnt = int(min<int64_t>(COLS, c1 - cb));
    const int kk = BF16 ? t : (t >> 1);
    const int64_t row = cb + min(kk, cnt - 1);
    if constexpr (BF16) {
      const u32x4* src = reinterpret_cast<const u32x4*>(Vhl + row * 32);
#pragma unroll
      for (int i = 0; i < NV; ++i) pv[i] = src[i];
    } else {
      const u32x4* src = reinterpret_cast<const u32x4*>(V + row * 16 + 8 * (t & 1));
#pragma unroll
      for (int i = 0; i < NV; ++i) pv[i] = src[i];
    }
    if constexpr (MX > 0) {
      const u32x4* src = reinterpret_cast<const u32x4*>(Vx + (cb + min(t & 127, cnt - 1)) * kKvMaxExact);
      px[0] = src[0];
      px[1] = src[1];
    }
  };
  auto store_v = [&](int cnt, const u32x4 (&pv)[NV], const u32x4 (&px)[2]) {
    if constexpr (BF16) {
      const bool ok = t < cnt;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t w = ok ? pv[i][e] : 0u;
          const int j = 8 * (i & 1) + 2 * e;  // halves 2e, 2e + 1 of piece i: columns j, j + 1
          if (i < 2) {
            vh[j][t] = uint16_t(w & 0xffffu);
            vh[j + 1][t] = uint16_t(w >> 16);
          } else {
            vl[j][t] = uint16_t(w & 0xffffu);
            vl[j + 1][t] = uint16_t(w >> 16);
          }
        }
    } else {
      const int kk = t >> 1, h = t & 1;
      const bool ok = kk < cnt;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) vs[8 * h + 4 * i + e][kk] = ok ? __uint_as_float(pv[i][e]) : 0.f;
    }
    if constexpr (MX > 0) {
      if (t < 128) {  // one thread per row of the stage
        const bool ok = t < cnt;
        const int slot = (t >> 3) * 10 + (t & 7);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const uint64_t lo = (uint64_t(px[i][1]) << 32) | px[i][0];
          const uint64_t hi = (uint64_t(px[i][3]) << 32) | px[i][2];
          vxs[2 * i][slot] = ok ? __longlong_as_double(int64_t(lo)) : 0.0;
          vxs[2 * i + 1][slot] = ok ? __longlong_as_double(int64_t(hi)) : 0.0;
        }
      }
    }
  };
  double acc64[4] = {0.0, 0.0, 0.0, 0.0};
  double accx[4][MX > 0 ? MX : 1];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
#pragma unroll
    for (int j = 0; j < (MX > 0 ? MX : 1); ++j) accx[rr][j] = 0.0;
  u32x4 pre[8], prev[NV], prex[2];
  if (c0 < c1) {
    load_stage(c0, pre);
    load_v(c0, prev, prex);
  }
  const int srow = 16 * wave + li;  // this lane's row in the tile (MFMA A operand)
  for (int64_t cb = c0; cb < c1; cb += COLS) {
    const int cnt = int(min<int64_t>(COLS, c1 - cb));
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q)
      *reinterpret_cast<u32x4*>(&ks[((q * 8 + tr) * KPAD + tc * PER) * ESZ]) = pre[q];
    store_v(cnt, prev, prex);
    __syncthreads();
    if (cb + COLS < c1) {
      load_stage(cb + COLS, pre);
      load_v(cb + COLS, prev, prex);
    }
    if (MX > 0) {  // exact columns: rows 4 (t/16) .. +3, columns [8 (t%16), 8 (t%16) + 8) of the stage
      const int xg = t >> 4, xs = t & 15;
      f32x4 kq[4][2];  // this thread's 4 x 8 block of the staged K
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const float* krow = reinterpret_cast<const float*>(ks) + (4 * xg + rr) * KPAD + xs * 8;
        kq[rr][0] = *reinterpret_cast<const f32x4*>(krow);
        kq[rr][1] = *reinterpret_cast<const f32x4*>(krow + 4);
      }
#pragma unroll
      for (int j = 0; j < (MX > 0 ? MX : 1); ++j) {
        double vx[8];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const double2 w = *reinterpret_cast<const double2*>(&vxs[j][xs * 10 + 2 * h]);
          vx[2 * h] = w.x;
          vx[2 * h + 1] = w.y;
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
          for (int e = 0; e < 8; ++e) accx[rr][j] = fma(double(kq[rr][e >> 2][e & 3]), vx[e], accx[rr][j]);
      }
    }
    f32x4 accA = {0.f, 0.f, 0.f, 0.f}, accB = {0.f, 0.f, 0.f, 0.f};
    if (BF16) {
      const uint16_t* arow = reinterpret_cast<const uint16_t*>(ks) + srow * KPAD + lg * QCOL;
#pragma unroll
      for (int kk = 0; kk < QCOL / 8; ++kk) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(arow + 8 * kk);
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&vh[li][lg * QCOL + 8 * kk]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&vl[li][lg * QCOL + 8 * kk]);
        accA = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, accA, 0, 0, 0);
        accB = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, accB, 0, 0, 0);
      }
    } else {
      const float* arow = reinterpret_cast<const float*>(ks) + srow * KPAD + lg * QCOL;
#pragma unroll
      for (int kk = 0; kk < QCOL / 4; ++kk) {
        const f32x4 a = *reinterpret_cast<const f32x4*>(arow + 4 * kk);
        const f32x4 b = *reinterpret_cast<const f32x4*>(&vs[li][lg * QCOL + 4 * kk]);
        accA = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], accA, 0, 0, 0);
        accB = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], accB, 0, 0, 0);
        accA = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], accA, 0, 0, 0);
        accB = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], accB, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[r] += double(accA[r]) + double(accB[r]);
  }
  const int64_t row0 = row_base + 16 * wave;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + 4 * lg + r;
    if (row < n) out[(int64_t(blockIdx.y) * n + row) * 16 + li] = acc64[r];
  }
  if (MX > 0) {  // the 16 column slices of a row group sit in adjacent lanes
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
      for (int j = 0; j < (MX > 0 ? MX : 1); ++j)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) accx[rr][j] += __shfl_xor(accx[rr][j], off);
    if ((t & 15) == 0) {
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int64_t row = row_base + 4 * (t >> 4) + rr;
        if (row < n) {
#pragma unroll
          for (int j = 0; j < (MX > 0 ? MX : 1); ++j)
            outx[(int64_t(blockIdx.y) * n + row) * kKvMaxExact + j] = accx[rr][j];
        }
      }
    }
  }
}

__global__ void kv_reduce_x_kernel(const double* __restrict__ part, int nseg, int64_t n, int mx, DstTable16 dst) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= n * 4) return;
  const int64_t i = t >> 2;
  const int j = int(t & 3);
  if (j >= mx) return;
  double s = 0.0;
  for (int k = 0; k < nseg; ++k) s += part[int64_t(k) * n * 4 + t];
  dst.p[j][i] = s;
}

// Vx[i][j] = src.p[j][i] for j < mx, 0 for mx <= j < 4
__global__ void kv_gather_x_kernel(SrcTable16 src, int mx, int64_t n, double* __restrict__ Vx) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= n * 4) return;
  const int64_t i = t >> 2;
  const int j = int(t & 3);
  Vx[t] = j < mx ? src.p[j][i] : 0.0;
}

// Vhl[i][j] = bf16(V[i][j]), Vhl[i][16 + j] = bf16(V[i][j] - that) (round to nearest even)
__global__ void kv_split_kernel(const float* __restrict__ V, int64_t n, uint16_t* __restrict__ Vhl) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= n * 16) return;
  const int64_t i = t >> 4;
  const int j = int(t & 15);
  const float val = V[t];
  const uint16_t h = f2bf(val);
  Vhl[i * 32 + j] = h;
  Vhl[i * 32 + 16 + j] = f2bf(val - __uint_as_float(uint32_t(h) << 16));
}

__global__ void kv_reduce_kernel(const double* __restrict__ part, int nseg, int64_t n, int m, double* __restrict__ U,
                                 int64_t ldu) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= n * 16) return;
  const int64_t i = t >> 4;
  const int j = int(t & 15);
  if (j >= m) return;
  double s = 0.0;
  for (int k = 0; k < nseg; ++k) s += part[int64_t(k) * n * 16 + t];
  U[i * ldu + j] = s;
}

namespace {
std::mutex g_kv_mu;
KvShape g_kv_shape[2][kKvBuckets];
bool g_kv_set[2][kKvBuckets] = {};
int kv_bucket(int64_t n) {
  int b = 0;
  while (b + 1 < kKvBuckets && (int64_t(4096) << b) < n) ++b;
  return b;
}
template <bool BF16>
void kv_launch(const KvShape& s, dim3 grid, const KMat& km, int64_t n, const float* V16, const uint16_t* Vhl,
               int64_t seg_cols, double* part, hipStream_t st) {
  if (s.nld == 0)
    kv_staged_kernel<BF16, 0><<<grid, 256, 0, st>>>(km.K, km.ld, n, n, V16, Vhl, seg_cols, part, nullptr, nullptr);
  else if (s.nld == 4 && s.prefetch)
    kv_mfma_kernel<BF16, 4, true><<<grid, 256, 0, st>>>(km.K, km.ld, n, n, V16, seg_cols, part);
  else if (s.nld == 4)
    kv_mfma_kernel<BF16, 4, false><<<grid, 256, 0, st>>>(km.K, km.ld, n, n, V16, seg_cols, part);
  else if (s.prefetch)
    kv_mfma_kernel<BF16, 8, true><<<grid, 256, 0, st>>>(km.K, km.ld, n, n, V16, seg_cols, part);
  else
    kv_mfma_kernel<BF16, 8, false><<<grid, 256, 0, st>>>(km.K, km.ld, n, n, V16, seg_cols, part);
}
}  // namespace

KvShape default_kv_shape(int dtype, int64_t n) {
  std::lock_guard<std::mutex> lk(g_kv_mu);
  const int d = dtype == KQR_BF16, b = kv_bucket(n);
  if (g_kv_set[d][b]) return g_kv_shape[d][b];
  return KvShape{};
}

void set_kv_shape(int dtype, int64_t n, KvShape s) {
  std::lock_guard<std::mutex> lk(g_kv_mu);
  const int d = dtype == KQR_BF16, b = kv_bucket(n);
  g_kv_shape[d][b] = s;
  g_kv_set[d][b] = true;
}

bool kv_shape_supported(const KvShape& s) {
  return (s.nld == 0 || s.nld == 4 || s.nld == 8) && s.segs >= 1 && s.segs <= kKvMaxSegs;
}

void kapply_kv(const KMat& km, int64_t n, const float* V16, int m, double* U, int64_t ldu, double* part,
               hipStream_t st, const KvShape* shape) {
  if (n <= 0) return;
  const KvShape s = shape ? *shape : default_kv_shape(km.dtype, n);
  if (!kv_shape_supported(s)) fail(KQR_EINVAL, "unsupported K V shape (nld %d, segs %d)", s.nld, s.segs);
  int segs = s.segs;
  int64_t seg_cols = (n + segs - 1) / segs;
  seg_cols = (seg_cols + kKC - 1) / kKC * kKC;
  segs = int((n + seg_cols - 1) / seg_cols);
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)segs);
  if (km.dtype == KQR_BF16) {
    // BF16 hi + lo parts of V, n x 32 halves, in the scratch past the segment partials
    uint16_t* Vhl = reinterpret_cast<uint16_t*>(part + size_t(kKvMaxSegs) * size_t(n) * 16);
    if (s.nld == 0) {
      kv_split_kernel<<<dim3((unsigned)((n * 16 + 255) / 256)), 256, 0, st>>>(V16, n, Vhl);
      KQR_LAUNCH_CHECK();
    }
    kv_launch<true>(s, grid, km, n, V16, Vhl, seg_cols, part, st);
  } else {
    kv_launch<false>(s, grid, km, n, V16, nullptr, seg_cols, part, st);
  }
  KQR_LAUNCH_CHECK();
  kv_reduce_kernel<<<dim3((unsigned)((n * 16 + 255) / 256)), 256, 0, st>>>(part, segs, n, m, U, ldu);
  KQR_LAUNCH_CHECK();
}

void kapply_kv_mixed(const KMat& km, int64_t n, const float* V16, int m, double* U, int64_t ldu, SrcTable16 xsrc,
                     int mx, DstTable16 xdst, double* part, hipStream_t st) {
  if (n <= 0) return;
  if (km.dtype != KQR_FP32 || km.layout != 0 || mx < 1 || mx > kKvMaxExact)
    fail(KQR_EINVAL, "exact columns need an FP32 K in the full layout and 1..%d of them", kKvMaxExact);
  int segs = default_kv_shape(km.dtype, n).segs;
  int64_t seg_cols = (n + segs - 1) / segs;
  seg_cols = (seg_cols + kKC - 1) / kKC * kKC;
  segs = int((n + seg_cols - 1) / seg_cols);
  // scratch: [segment partials 16 n][BF16 V parts 16 n] per kv_scratch_doubles, then
  // [exact partials kKvMaxSegs 4 n][Vx 4 n]
  double* partx = part + (size_t(kKvMaxSegs) + 1) * size_t(n) * 16;
  double* Vx = partx + size_t(kKvMaxSegs) * size_t(n) * 4;
  kv_gather_x_kernel<<<dim3((unsigned)((n * 4 + 255) / 256)), 256, 0, st>>>(xsrc, mx, n, Vx);
  KQR_LAUNCH_CHECK();
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)segs);
  // FP64 work for the exact columns asked for (1, 2 or 4): fewer columns, fewer registers
  if (mx == 1)
    kv_staged_kernel<false, 1><<<grid, 256, 0, st>>>(km.K, km.ld, n, n, V16, nullptr, seg_cols, part, Vx, partx);
  else if (mx == 2)
    kv_staged_kernel<false, 2><<<grid, 256, 0, st>>>(km.K, km.ld, n, n, V16, nullptr, seg_cols, part, Vx, partx);
  else
    kv_staged_kernel<false, kKvMaxExact><<<grid, 256, 0, st>>>(km.K, km.ld, n, n, V16, nullptr, seg_cols, part, Vx,
                                                                 partx);
  KQR_LAUNCH_CHECK();
  if (m > 0) {
    kv_reduce_kernel<<<dim3((unsigned)((n * 16 + 255) / 256)), 256, 0, st>>>(part, segs, n, m, U, ldu);
    KQR_LAUNCH_CHECK();
  }
  kv_reduce_x_kernel<<<dim3((unsigned)((n * 4 + 255) / 256)), 256, 0, st>>>(partx, segs, n, mx, xdst);
  KQR_LAUNCH_CHECK();
}

// V16[i][j] = float(src_j[i]) for j < m, 0 for m <= j < 16 (rows < n_pad; rows >= n are 0)
__global__ void kv_gather_kernel(SrcTable16 src, int m, int64_t n, int64_t n_pad, float* __restrict__ V16) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= n_pad * 16) return;
  const int64_t i = t >> 4;
  const int j = int(t & 15);
  V16[t] = (j < m && i < n) ? float(src.p[j][i]) : 0.f;
}

// dst_j[i] = U[i][j]
__global__ void kv_scatter_kernel(const double* __restrict__ U, int m, int64_t n, DstTable16 dst) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= n * 16) return;
  const int64_t i = t >> 4;
  const int j = int(t & 15);
  if (j < m) dst.p[j][i] = U[t];
}

__global__ void kv_gather_strided_kernel(const double* __restrict__ V, int64_t ldv, int m, int64_t n, int64_t n_pad,
                                         float* __restrict__ V16) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= n_pad * 16) return;
  const int64_t i = t >> 4;
  const int j = int(t & 15);
  V16[t] = (j < m && i < n) ? float(V[i * ldv + j]) : 0.f;
}

void kv_gather_strided(const double* V, int64_t ldv, int m, int64_t n, int64_t n_pad, float* V16, hipStream_t st) {
  kv_gather_strided_kernel<<<dim3((unsigned)((n_pad * 16 + 255) / 256)), 256, 0, st>>>(V, ldv, m, n, n_pad, V16);
  KQR_LAUNCH_CHECK();
}

void kv_gather(SrcTable16 src, int m, int64_t n, int64_t n_pad, float* V16, hipStream_t st) {
  kv_gather_kernel<<<dim3((unsigned)((n_pad * 16 + 255) / 256)), 256, 0, st>>>(src, m, n, n_pad, V16);
  KQR_LAUNCH_CHECK();
}

void kv_scatter(const double* U16, int m, int64_t n, DstTable16 dst, hipStream_t st) {
  kv_scatter_kernel<<<dim3((unsigned)((n * 16 + 255) / 256)), 256, 0, st>>>(U16, m, n, dst);
  KQR_LAUNCH_CHECK();
}

// ----------------------------------------------------------------- many problems, one launch
// Rows [row0, row0 + 8) of task tk, one wave: u = K v with v rounded to FP32
// (as every fast apply rounds v), FP32 products within a 16-byte chunk, FP64
// sums across chunks and lanes.
__device__ __forceinline__ void problem_rows(const ProblemTask& tk, int64_t row0, int lane) {
  constexpr int ROWS = 8;
  const bool bf = tk.dtype == KQR_BF16;
  const int vec = bf ? 8 : 4;
  const int64_t nchunk = tk.n / vec;
  double acc[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) acc[r] = 0.0;
  const char* base = static_cast<const char*>(tk.K);
  const int64_t rstride = tk.ld * (bf ? 2 : 4);
  for (int64_t c = lane; c < nchunk; c += 64) {
    float vv[8];
    const double* vp = tk.v + c * vec;  // 8-byte loads: v may sit at any double offset
#pragma unroll
    for (int e = 0; e < 4; ++e) vv[e] = float(vp[e]);
    if (bf) {
#pragma unroll
      for (int e = 4; e < 8; ++e) vv[e] = float(vp[e]);
    }
    u32x4 kk[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const int64_t rr = min(row0 + r, tk.n - 1);
      kk[r] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(base + rr * rstride) + c);
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      float a = 0.f;
      if (bf) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t w = kk[r][e >> 1];
          a = fmaf(__uint_as_float((e & 1) ? (w & 0xffff0000u) : (w << 16)), vv[e], a);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) a = fmaf(__uint_as_float(kk[r][e]), vv[e], a);
      }
      acc[r] += double(a);
    }
  }
  const int64_t col = nchunk * vec + lane;
  if (col < tk.n) {
    const double ve = double(float(tk.v[col]));
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const int64_t rr = min(row0 + r, tk.n - 1);
      const float ke = bf ? __uint_as_float(uint32_t(reinterpret_cast<const uint16_t*>(base + rr * rstride)[col]) << 16)
                          : reinterpret_cast<const float*>(base + rr * rstride)[col];
      acc[r] = fma(double(ke), ve, acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < ROWS; ++r)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
#pragma unroll
  for (int r = 0; r < ROWS; ++r)
    if (lane == r && row0 + r < tk.n) tk.u[row0 + r] = acc[r];
}

// Persistent launch: every workgroup takes items (32-row blocks: 4 waves of
// 8 rows) from a counter until the items run out.  Items are numbered in task
// order (first_block = exclusive prefix of the tasks' block counts).  Eight
// counters, one per XCD (workgroups are dealt to the XCDs round-robin in
// blockIdx order): counter x hands out the items x, x + 8, x + 16, ..., so
// each XCD still sees an even share of the largest-first order, and the
// atomics on one address (a few tens of nanoseconds apart at best) are an
// eighth as many.  The counters are never reset: counter x's items in this
// launch are its values [base_x, base_x + items_x), and each workgroup on it
// takes exactly one value beyond them before it stops, so the next launch
// starts at base_x + items_x + (workgroups on counter x).
struct QueueBases {
  unsigned long long b[kQueueCounters];
};

__global__ __launch_bounds__(256) void kapply_problems_queue_kernel(const ProblemTask* __restrict__ tasks, int ntasks,
                                                                    const int* __restrict__ first_block, int total,
                                                                    unsigned long long* __restrict__ ctr,
                                                                    QueueBases base) {
  __shared__ int item_sh;
  const int lane = threadIdx.x & 63;
  const int x = int(blockIdx.x % kQueueCounters);
  for (;;) {
    if (threadIdx.x == 0) {
      const long long k = (long long)(atomicAdd(ctr + x, 1ull) - base.b[x]);
      item_sh = k < 0 ? -1 : int(min<long long>(k * kQueueCounters + x, total));
    }
    __syncthreads();
    const int item = item_sh;
    __syncthreads();  // every wave has the item before thread 0 takes the next
    if (item < 0 || item >= total) break;  // (negative only if launches of one queue overlapped)
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first_block[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    const ProblemTask tk = tasks[lo];
    const int64_t row0 = (int64_t(item - first_block[lo]) * 4 + (threadIdx.x >> 6)) * 8;
    if (row0 < tk.n) problem_rows(tk, row0, lane);
  }
}

int problem_blocks(int64_t n) { return int((n + 31) / 32); }

namespace {
size_t queue_table_bytes(size_t cap) {
  return (cap * sizeof(ProblemTask) + (cap + 1) * sizeof(int) + 255) / 256 * 256;
}
}  // namespace

ProblemQueue::ProblemQueue(size_t max_tasks)
    : cap_(std::max<size_t>(max_tasks, 1)), slot_bytes_(queue_table_bytes(cap_)), table_(kRing * slot_bytes_),
      stage_(kRing * slot_bytes_), ctr_(kQueueCounters * sizeof(unsigned long long)) {
  KQR_CHECK_HIP(hipMemset(ctr_.ptr, 0, kQueueCounters * sizeof(unsigned long long)));
  for (auto& e : copied_) KQR_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

ProblemQueue::~ProblemQueue() {
  for (auto& e : copied_) (void)hipEventDestroy(e);
}

void ProblemQueue::launch(const std::vector<ProblemTask>& tasks, hipStream_t st) {
  if (tasks.empty()) return;
  if (tasks.size() > cap_) fail(KQR_EHIP, "internal: %zu tasks for a queue of %zu", tasks.size(), cap_);
  const int k = next_;
  next_ = (next_ + 1) % kRing;
  // the staging copy of this ring slot was last read by the copy recorded kRing launches ago
  if (used_[k]) KQR_CHECK_HIP(hipEventSynchronize(copied_[k]));
  char* stage = static_cast<char*>(stage_.ptr) + size_t(k) * slot_bytes_;
  char* table = static_cast<char*>(table_.ptr) + size_t(k) * slot_bytes_;
  const size_t ntask = tasks.size();
  memcpy(stage, tasks.data(), ntask * sizeof(ProblemTask));
  int* first = reinterpret_cast<int*>(stage + ntask * sizeof(ProblemTask));
  int total = 0;
  for (size_t t = 0; t < ntask; ++t) {
    first[t] = total;
    total += problem_blocks(tasks[t].n);
  }
  first[ntask] = total;
  const size_t bytes = ntask * sizeof(ProblemTask) + (ntask + 1) * sizeof(int);
  KQR_CHECK_HIP(hipMemcpyAsync(table, stage, bytes, hipMemcpyHostToDevice, st));
  KQR_CHECK_HIP(hipEventRecord(copied_[k], st));
  used_[k] = true;
  const int grid = std::min(total, kQueueWgs);
  QueueBases qb;
  for (int x = 0; x < kQueueCounters; ++x) qb.b[x] = base_[x];
  kapply_problems_queue_kernel<<<grid, 256, 0, st>>>(
      reinterpret_cast<const ProblemTask*>(table), int(ntask),
      reinterpret_cast<const int*>(table + ntask * sizeof(ProblemTask)), total, ctr_.as<unsigned long long>(), qb);
  KQR_LAUNCH_CHECK();
  for (int x = 0; x < kQueueCounters; ++x) {
    const uint64_t items = x < total ? uint64_t((total - x + kQueueCounters - 1) / kQueueCounters) : 0;
    const uint64_t wgs = x < grid ? uint64_t((grid - x + kQueueCounters - 1) / kQueueCounters) : 0;
    base_[x] += items + wgs;
  }
}

}  // namespace kqr
