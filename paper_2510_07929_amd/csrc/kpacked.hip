// Symmetric K stored once: the upper triangle in square tiles.
//
// K is symmetric (Section 1: k(x, x') = k(x', x)), so only the tiles (I, J)
// with I <= J of a tiling by kPkT x kPkT blocks are stored, tile-row by
// tile-row: tile (I, J) sits at tile index I nt - I (I - 1) / 2 + (J - I),
// nt = ceil(n / kPkT), each tile row-major and zero beyond n.  A K-apply then
// streams about n^2 / 2 entries instead of n^2: every off-diagonal tile feeds
// its rows (K_IJ v_J) and its columns (K_IJ^T v_I).
#include "kernel_entry.h"
#include "kqr_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

namespace kqr {

namespace {

typedef uint32_t pk_u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t pk_to_bf16(float f) {  // round to nearest even (finite entries)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

template <bool BF16>
__device__ __forceinline__ float pk_elem(const pk_u32x4& w, int e) {
  if (BF16) {
    const uint32_t word = w[e >> 1];
    return __uint_as_float((e & 1) ? (word & 0xffff0000u) : (word << 16));
  }
  return __uint_as_float(w[e]);
}

}  // namespace

int64_t packed_tile_count(int64_t n) {
  const int64_t nt = (n + kPkT - 1) / kPkT;
  return nt * (nt + 1) / 2;
}

int64_t packed_tiles_per_side(int64_t n) { return (n + kPkT - 1) / kPkT; }

size_t packed_bytes(int64_t n, int dtype) {
  return size_t(packed_tile_count(n)) * kPkT * kPkT * (dtype == KQR_BF16 ? 2 : 4);
}

// ================================================================= build
// One workgroup per tile: 256 threads, each thread one column of the tile and
// half of its rows; the tile's rows of X and their norms staged in LDS.
template <int PMAX, bool LAP, bool BF16>
__global__ __launch_bounds__(256) void kbuild_packed_kernel(const float* __restrict__ X, const float* __restrict__ q,
                                                            int64_t n, int p, int64_t nt, float ng,
                                                            void* __restrict__ Kout) {
  __shared__ float xs[kPkT][PMAX];
  __shared__ float qs[kPkT];
  // tile (I, J) from the linear tile index (row I holds nt - I tiles)
  const int64_t t = blockIdx.x;
  int64_t I = 0, first = 0;
  {
    int64_t lo = 0, hi = nt - 1;  // largest I with pk_tile_index(I, I, nt) <= t
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (pk_tile_index(mid, mid, nt) <= t) lo = mid;
      else hi = mid - 1;
    }
    I = lo;
    first = pk_tile_index(I, I, nt);
  }
  const int64_t J = I + (t - first);
  for (int e = threadIdx.x; e < kPkT * PMAX; e += 256) {
    const int r = e / PMAX, k = e % PMAX;
    const int64_t i = I * kPkT + r;
    xs[r][k] = (i < n && k < p) ? X[i * p + k] : 0.f;
  }
  for (int r = threadIdx.x; r < kPkT; r += 256) {
    const int64_t i = I * kPkT + r;
    qs[r] = (i < n && !LAP) ? q[i] : 0.f;
  }
  __syncthreads();
  const int c = threadIdx.x % kPkT;
  const int r0 = threadIdx.x / kPkT;  // 0 or 1: even or odd rows
  const int64_t j = J * kPkT + c;
  const bool valid = j < n;
  float xj[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) xj[k] = (valid && k < p) ? X[j * p + k] : 0.f;
  const float qj = (valid && !LAP) ? q[j] : 0.f;
  const size_t base = size_t(t) * kPkT * kPkT;
  for (int r = r0; r < kPkT; r += 2) {
    const int64_t i = I * kPkT + r;
    float val = 0.f;
    if (valid && i < n) {
      float d = pair_dist<PMAX, LAP>(xs[r], qs[r], xj, qj);
      if (i == j) d = 0.f;
      val = kexp2(ng * d);
    }
    const size_t off = base + size_t(r) * kPkT + c;
    if (BF16) __builtin_nontemporal_store(pk_to_bf16(val), static_cast<uint16_t*>(Kout) + off);
    else __builtin_nontemporal_store(val, static_cast<float*>(Kout) + off);
  }
}

template <int PMAX>
static void kbuild_packed_p(const float* X, const float* q, int64_t n, int p, KernelSpec ks, int dtype, void* K,
                            hipStream_t st) {
  const int64_t nt = (n + kPkT - 1) / kPkT;
  const dim3 grid((unsigned)packed_tile_count(n));
  const float ng = -float(ks.gamma) * kLog2e;
  const bool lap = ks.kind == KQR_LAPLACIAN, bf = dtype == KQR_BF16;
  if (lap && bf) kbuild_packed_kernel<PMAX, true, true><<<grid, 256, 0, st>>>(X, q, n, p, nt, ng, K);
  else if (lap) kbuild_packed_kernel<PMAX, true, false><<<grid, 256, 0, st>>>(X, q, n, p, nt, ng, K);
  else if (bf) kbuild_packed_kernel<PMAX, false, true><<<grid, 256, 0, st>>>(X, q, n, p, nt, ng, K);
  else kbuild_packed_kernel<PMAX, false, false><<<grid, 256, 0, st>>>(X, q, n, p, nt, ng, K);
  KQR_LAUNCH_CHECK();
}

void kbuild_packed(const float* X, const float* sqn, int64_t n, int p, KernelSpec ks, int dtype, void* K,
                   hipStream_t st) {
  if (n <= 0) return;
  // RBF with p <= 32: the Gram term on the matrix cores, entries as in the full layout
  if (kbuild_mfma(X, sqn, n, p, ks, dtype, K, packed_tiles_per_side(n), 1, st)) return;
  if (p <= 8) kbuild_packed_p<8>(X, sqn, n, p, ks, dtype, K, st);
  else if (p <= 16) kbuild_packed_p<16>(X, sqn, n, p, ks, dtype, K, st);
  else if (p <= 32) kbuild_packed_p<32>(X, sqn, n, p, ks, dtype, K, st);
  else if (p <= 64) kbuild_packed_p<64>(X, sqn, n, p, ks, dtype, K, st);
  else fail(KQR_EINVAL, "feature dimension p=%d exceeds 64", p);
}

// ================================================================= apply
// Workgroup b walks strip k of tile-row I (b -> (I, k) by pk_strip_coords),
// the tiles J = I + k*strip ...; every off-diagonal tile feeds its rows (K_IJ v_J) and its columns
// (K_IJ^T v_I).  Row sums stay in registers across the strip (the same rows
// of every tile), column sums are written as one partial per tile.  Thread
// mappings (tuned per dtype):
//   rows map (0: 256 threads, 2: 512 threads, half the loads per lane and
//     per tile): LPR lanes read one tile row contiguously (512 B FP32, 256 B
//     BF16); column sums are reduced across the row groups in LDS, the
//     reduction of tile J deferred until the loads of tile J+1 are in flight
//     (double-buffered LDS, one barrier per tile);
//   cols map (1): wave w owns 32 columns of every tile; column sums need only
//     shuffles inside the wave, row sums are combined across waves at the
//     end of the strip.
//   fast  (EXACT=false): v in FP32, FP32 products summed in FP32 within a
//                        16-byte chunk (rows) or a tile (columns), FP64 beyond;
//   exact (EXACT=true) : v in FP64, products and sums in FP64.
template <bool BF16, bool EXACT, int NT>
__global__ __launch_bounds__(NT) void kapply_packed_rows_kernel(const void* __restrict__ Kp, int64_t n, int64_t nt,
                                                                int strip, int64_t nsx, const float* __restrict__ v32,
                                                                const double* __restrict__ v64,
                                                                double* __restrict__ rowpart,
                                                                double* __restrict__ colpart, int64_t nstrips) {
  constexpr int VEC = BF16 ? 8 : 4;     // entries per 16-byte load
  constexpr int LPR = kPkT / VEC;       // lanes per tile row (32 or 16)
  constexpr int RPS = NT / LPR;         // rows per step
  constexpr int STEPS = kPkT / RPS;     // loads in flight per lane per tile
  constexpr int ESZ = BF16 ? 2 : 4;
  typedef typename std::conditional<EXACT, double, float>::type acc_t;
  __shared__ acc_t cs[2][RPS][kPkT + 1];

  // one strip per workgroup, or (persistent launch) strips b, b + gridDim.x, ...
  for (int64_t sb = blockIdx.x; sb < nstrips; sb += gridDim.x) {
  int64_t I, kstrip;
  pk_strip_coords(sb, nt, strip, I, kstrip);
  const int64_t J0 = I + kstrip * strip;
  const int64_t J1 = std::min<int64_t>(nt, J0 + strip);
  const int tid = threadIdx.x;
  const int cl = tid % LPR, rg = tid / LPR;

  acc_t vi[STEPS];
#pragma unroll
  for (int s = 0; s < STEPS; ++s) {
    const int64_t row = I * kPkT + rg + RPS * s;
    vi[s] = row < n ? (EXACT ? acc_t(v64[row]) : acc_t(v32[row])) : acc_t(0);
  }
  double racc[STEPS];
#pragma unroll
  for (int s = 0; s < STEPS; ++s) racc[s] = 0.0;

  // column partial of tile `tix` from LDS buffer b (all row groups written)
  auto flush_cols = [&](int b, int64_t tix) {
    if (tid < kPkT) {
      double sum = 0.0;
#pragma unroll
      for (int g = 0; g < RPS; ++g) sum += double(cs[b][g][tid]);
      colpart[size_t(tix) * kPkT + tid] = sum;
    }
  };
  int buf = 0;
  int64_t pending = -1;  // tile whose column sums wait in cs[buf ^ 1]
  for (int64_t J = J0; J < J1; ++J) {
    const int64_t tix = pk_tile_index(I, J, nt);
    const pk_u32x4* tile =
        reinterpret_cast<const pk_u32x4*>(static_cast<const char*>(Kp) + size_t(tix) * kPkT * kPkT * ESZ);
    pk_u32x4 kk[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) kk[s] = __builtin_nontemporal_load(tile + (rg + RPS * s) * LPR + cl);
    acc_t vj[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t col = J * kPkT + cl * VEC + e;
      vj[e] = col < n ? (EXACT ? acc_t(v64[col]) : acc_t(v32[col])) : acc_t(0);
    }
    if (pending >= 0) {  // previous tile's column sums, while this tile's loads are in flight
      __syncthreads();
      flush_cols(buf ^ 1, pending);
      pending = -1;
    }
    acc_t cacc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) cacc[e] = acc_t(0);
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      acc_t r = acc_t(0);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const acc_t ke = acc_t(pk_elem<BF16>(kk[s], e));
        r = fma(ke, vj[e], r);
        cacc[e] = fma(ke, vi[s], cacc[e]);
      }
      racc[s] += double(r);
    }
    if (J != I) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) cs[buf][rg][cl * VEC + e] = cacc[e];
      pending = tix;
      buf ^= 1;
    }
  }
  if (pending >= 0) {
    __syncthreads();
    flush_cols(buf ^ 1, pending);
  }
  // row sums: the LPR lanes of a row are contiguous inside one wave
#pragma unroll
  for (int s = 0; s < STEPS; ++s)
#pragma unroll
    for (int off = LPR / 2; off >= 1; off >>= 1) racc[s] += __shfl_xor(racc[s], off);
  if (cl == 0) {
    double* rp = rowpart + (size_t(I) * nsx + kstrip) * kPkT;
#pragma unroll
    for (int s = 0; s < STEPS; ++s) rp[rg + RPS * s] = racc[s];
  }
  __syncthreads();  // LDS of this strip read by every thread before the next strip writes it
  }
}

template <bool BF16, bool EXACT>
__global__ __launch_bounds__(256) void kapply_packed_cols_kernel(const void* __restrict__ Kp, int64_t n, int64_t nt,
                                                            int strip, int64_t nsx, const float* __restrict__ v32,
                                                            const double* __restrict__ v64,
                                                            double* __restrict__ rowpart,
                                                            double* __restrict__ colpart) {
  constexpr int VEC = BF16 ? 8 : 4;     // entries per 16-byte load
  constexpr int CPW = kPkT / 4;         // columns per wave
  constexpr int LPW = CPW / VEC;        // lanes per row segment (8 or 4)
  constexpr int RPS = 64 / LPW;         // rows per wave step (8 or 16)
  constexpr int STEPS = kPkT / RPS;     // 16 or 8
  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int CHUNKS_PER_ROW = kPkT / VEC;  // 16-byte chunks in a tile row
  typedef typename std::conditional<EXACT, double, float>::type acc_t;
  __shared__ double rs_lds[4][kPkT];

  int64_t I, kstrip;
  pk_strip_coords(blockIdx.x, nt, strip, I, kstrip);
  const int64_t J0 = I + kstrip * strip;
  const int64_t J1 = std::min<int64_t>(nt, J0 + strip);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane % LPW, g = lane / LPW;
  const int chunk = w * LPW + c;  // this lane's 16-byte chunk within a tile row

  acc_t vi[STEPS];
#pragma unroll
  for (int s = 0; s < STEPS; ++s) {
    const int64_t row = I * kPkT + g + RPS * s;
    vi[s] = row < n ? (EXACT ? acc_t(v64[row]) : acc_t(v32[row])) : acc_t(0);
  }
  double racc[STEPS];
#pragma unroll
  for (int s = 0; s < STEPS; ++s) racc[s] = 0.0;

  for (int64_t J = J0; J < J1; ++J) {
    const int64_t tix = pk_tile_index(I, J, nt);
    const pk_u32x4* tile =
        reinterpret_cast<const pk_u32x4*>(static_cast<const char*>(Kp) + size_t(tix) * kPkT * kPkT * ESZ);
    pk_u32x4 kk[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) kk[s] = __builtin_nontemporal_load(tile + (g + RPS * s) * CHUNKS_PER_ROW + chunk);
    acc_t vj[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t col = J * kPkT + chunk * VEC + e;
      vj[e] = col < n ? (EXACT ? acc_t(v64[col]) : acc_t(v32[col])) : acc_t(0);
    }
    acc_t cacc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) cacc[e] = acc_t(0);
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      acc_t r = acc_t(0);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const acc_t ke = acc_t(pk_elem<BF16>(kk[s], e));
        r = fma(ke, vj[e], r);
        cacc[e] = fma(ke, vi[s], cacc[e]);
      }
      racc[s] += double(r);
    }
    if (J != I) {  // column sums of an off-diagonal tile: across the RPS row groups of the wave
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        double t = double(cacc[e]);
#pragma unroll
        for (int off = LPW; off < 64; off <<= 1) t += __shfl_xor(t, off);
        if (g == 0) colpart[size_t(tix) * kPkT + chunk * VEC + e] = t;
      }
    }
  }
  // row sums: across the LPW lanes of a segment, then across the four waves
#pragma unroll
  for (int s = 0; s < STEPS; ++s) {
#pragma unroll
    for (int off = 1; off < LPW; off <<= 1) racc[s] += __shfl_xor(racc[s], off);
    if (c == 0) rs_lds[w][g + RPS * s] = racc[s];
  }
  __syncthreads();
  if (threadIdx.x < kPkT) {
    const int r = threadIdx.x;
    rowpart[(size_t(I) * nsx + kstrip) * kPkT + r] = ((rs_lds[0][r] + rs_lds[1][r]) + rs_lds[2][r]) + rs_lds[3][r];
  }
}

// Square blocks of B x B tiles (maps 4 and 5): workgroup b takes block
// (BI, BJ), BJ >= BI, of the upper triangle of the block grid (nb =
// ceil(nt / B) blocks per side) -- tile-rows I = BI B ..  BI B + B - 1 against
// tile-columns J = BJ B .. BJ B + B - 1, J >= I.  Inside a tile, map 4 gives
// each wave 32 columns of all 128 rows (CW = 4 waves across), map 5 (WIDE)
// 64 columns of 64 rows (CW = 2 across, RW = 2 down): with BF16 entries a
// 64-column row segment is a whole 128-byte line, where the 32-column form
// reads each line in halves from two waves.  LPW lanes cover a wave's row
// segment, RPS row groups its rows.  Row sums are finished once per tile-row
// of the block, across lanes and waves through LDS; column sums stay in FP64
// per lane across the block's tile-rows and are reduced inside the wave at
// the end of the block (and, for map 5, across the two waves down the rows
// through LDS).  So a block writes B row partials and B column partials for
// B^2 tiles, where a strip writes a column partial for every tile: those
// writes, mixed into the read stream, are what held the strip maps back.
//   rowpart: (I nb + BJ) kPkT + r   (the row sums of tile-row I in block column BJ)
//   colpart: (BI nt + J) kPkT + c   (the column sums of tile-column J in block row BI)
template <int CTRL>
__device__ __forceinline__ double pk_dpp(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(u)), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

// x + the value of the lane 16 (SWAP16) or 32 lanes away, the same on both lanes
template <bool SWAP16>
__device__ __forceinline__ double pk_swap_sum(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t l = uint32_t(u), h = uint32_t(u >> 32);
  uint32_t l0, l1, h0, h1;
  if constexpr (SWAP16) {
    const auto a = __builtin_amdgcn_permlane16_swap(l, l, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(h, h, false, false);
    l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
  } else {
    const auto a = __builtin_amdgcn_permlane32_swap(l, l, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(h, h, false, false);
    l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
  }
  return __builtin_bit_cast(double, (uint64_t(h0) << 32) | l0) + __builtin_bit_cast(double, (uint64_t(h1) << 32) | l1);
}

template <bool BF16, bool EXACT, int B, bool WIDE>
__global__ __launch_bounds__(256) void kapply_packed_blocks_kernel(const void* __restrict__ Kp, int64_t n,
                                                                   int64_t nt, int64_t nb,
                                                                   const float* __restrict__ v32,
                                                                   const double* __restrict__ v64,
                                                                   double* __restrict__ rowpart,
                                                                   double* __restrict__ colpart) {
  constexpr int VEC = BF16 ? 8 : 4;     // entries per 16-byte load
  constexpr int CW = WIDE ? 2 : 4;      // waves across a tile's columns
  constexpr int RW = 4 / CW;            // waves down its rows
  constexpr int LPW = kPkT / CW / VEC;  // lanes per row segment of a wave's columns
  constexpr int RPS = 64 / LPW;         // rows per wave step
  constexpr int STEPS = kPkT / RW / RPS;
  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int CHUNKS_PER_ROW = kPkT / VEC;
  constexpr int NPART = CW * LPW;       // row partials per row (lanes c of the waves sharing the rows)
  typedef typename std::conditional<EXACT, double, float>::type acc_t;
  __shared__ double rs[NPART][kPkT + 1];
  __shared__ double cs2[RW > 1 ? RW : 1][RW > 1 ? B : 1][kPkT];

  const int64_t b = blockIdx.x;
  int64_t BI = 0;
  {
    int64_t lo = 0, hi = nb - 1;  // largest BI whose first block is <= b
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (pk_tile_index(mid, mid, nb) <= b) lo = mid;
      else hi = mid - 1;
    }
    BI = lo;
  }
  const int64_t BJ = BI + (b - pk_tile_index(BI, BI, nb));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane % LPW, g = lane / LPW;
  const int cw = w % CW, rw = w / CW;
  const int chunk = cw * LPW + c;  // this lane's 16-byte chunk within a tile row
  const int row0 = rw * (kPkT / RW) + g;  // this lane's rows: row0 + RPS s

  acc_t vj[B][VEC];
#pragma unroll
  for (int jj = 0; jj < B; ++jj)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t col = (BJ * B + jj) * kPkT + chunk * VEC + e;
      vj[jj][e] = col < n ? (EXACT ? acc_t(v64[col]) : acc_t(v32[col])) : acc_t(0);
    }
  double cold[B][VEC];
#pragma unroll
  for (int jj = 0; jj < B; ++jj)
#pragma unroll
    for (int e = 0; e < VEC; ++e) cold[jj][e] = 0.0;

  for (int ii = 0; ii < B; ++ii) {
    const int64_t I = BI * B + ii;
    if (I >= nt) break;  // the same for the whole workgroup
    acc_t vi[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      const int64_t row = I * kPkT + row0 + RPS * s;
      vi[s] = row < n ? (EXACT ? acc_t(v64[row]) : acc_t(v32[row])) : acc_t(0);
    }
    double racc[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) racc[s] = 0.0;
#pragma unroll
    for (int jj = 0; jj < B; ++jj) {
      const int64_t J = BJ * B + jj;
      if (J < I || J >= nt) continue;  // the same for the whole workgroup
      const pk_u32x4* tile = reinterpret_cast<const pk_u32x4*>(static_cast<const char*>(Kp) +
                                                               size_t(pk_tile_index(I, J, nt)) * kPkT * kPkT * ESZ);
      pk_u32x4 kk[STEPS];
#pragma unroll
      for (int s = 0; s < STEPS; ++s) kk[s] = __builtin_nontemporal_load(tile + (row0 + RPS * s) * CHUNKS_PER_ROW + chunk);
      acc_t cacc[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) cacc[e] = acc_t(0);
#pragma unroll
      for (int s = 0; s < STEPS; ++s) {
        acc_t r = acc_t(0);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const acc_t ke = acc_t(pk_elem<BF16>(kk[s], e));
          r = fma(ke, vj[jj][e], r);
          cacc[e] = fma(ke, vi[s], cacc[e]);
        }
        racc[s] += double(r);
      }
      if (J != I) {  // the diagonal tile feeds its rows only
#pragma unroll
        for (int e = 0; e < VEC; ++e) cold[jj][e] += double(cacc[e]);
      }
    }
    // row sums of tile-row I: partials of row row0 + RPS s in lanes c of the waves sharing it
#pragma unroll
    for (int s = 0; s < STEPS; ++s) rs[cw * LPW + c][row0 + RPS * s] = racc[s];
    __syncthreads();
    {
      const int row = threadIdx.x >> 1, half = threadIdx.x & 1;
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < NPART / 2; ++k) t += rs[half * (NPART / 2) + k][row];
      t += pk_dpp<0xB1>(t);  // quad_perm [1, 0, 3, 2]: the other half of the row
      if (half == 0) rowpart[(size_t(I) * nb + BJ) * kPkT + row] = t;
    }
    __syncthreads();  // rs is rewritten by the next tile-row
  }
  // column sums: across the RPS row groups of the wave (lane bits above c),
  // then (RW = 2) across the two waves down the rows, through LDS
#pragma unroll
  for (int jj = 0; jj < B; ++jj) {
    const int64_t J = BJ * B + jj;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      double t = cold[jj][e];
      if (LPW <= 4) t += pk_dpp<0x124>(t);  // row_ror:4
      if (LPW <= 8) t += pk_dpp<0x128>(t);  // row_ror:8
      t = pk_swap_sum<true>(t);
      t = pk_swap_sum<false>(t);
      if (RW == 1) {
        if (g == 0 && J < nt) colpart[(size_t(BI) * nt + J) * kPkT + chunk * VEC + e] = t;
      } else if (g == 0) {
        cs2[rw][jj][chunk * VEC + e] = t;
      }
    }
  }
  if (RW > 1) {
    __syncthreads();
    for (int k = threadIdx.x; k < B * kPkT; k += 256) {
      const int jj = k / kPkT, col = k % kPkT;
      const int64_t J = BJ * B + jj;
      if (J < nt) colpart[(size_t(BI) * nt + J) * kPkT + col] = cs2[0][jj][col] + cs2[RW > 1 ? 1 : 0][jj][col];
    }
  }
}

// u_T = the row partials of tile-row T (block columns BT .. nb - 1), then the
// column partials of tile-column T (block rows 0 .. BT), BT = T / B, each
// split over four thread groups added in a fixed order.
__global__ __launch_bounds__(kPkT * 4) void packed_reduce_blocks_kernel(const double* __restrict__ rowpart,
                                                                       const double* __restrict__ colpart,
                                                                       int64_t n, int64_t nt, int64_t nb, int B,
                                                                       double* __restrict__ u, int64_t ldu) {
  __shared__ double part[4][kPkT];
  const int64_t T = blockIdx.x;
  const int r = threadIdx.x % kPkT, h = threadIdx.x / kPkT;
  const int64_t BT = T / B;
  const int64_t nrow = nb - BT;
  const int64_t nterm = nrow + BT + 1;
  double s = 0.0;
  for (int64_t k = h; k < nterm; k += 4)
    s += k < nrow ? rowpart[(size_t(T) * nb + BT + k) * kPkT + r] : colpart[(size_t(k - nrow) * nt + T) * kPkT + r];
  part[h][r] = s;
  __syncthreads();
  const int64_t i = T * kPkT + r;
  if (h == 0 && i < n) u[i * ldu] = ((part[0][r] + part[1][r]) + part[2][r]) + part[3][r];
}

// u_i = sum of the strip partials of i's tile-row, then the column partials of
// the tiles above i's diagonal tile, in that fixed order.  Block I covers the
// rows of tile-row I with kRedSplit threads per row, each summing every
// kRedSplit-th term; the split sums are added in a fixed order.
constexpr int kRedSplit = 4;
__global__ __launch_bounds__(kPkT * kRedSplit) void packed_reduce_kernel(
    const double* __restrict__ rowpart, const double* __restrict__ colpart, int64_t n, int64_t nt, int strip,
    int64_t nsx, double* __restrict__ u, int64_t ldu) {
  __shared__ double part[kRedSplit][kPkT];
  const int64_t I = blockIdx.x;
  const int r = threadIdx.x % kPkT, h = threadIdx.x / kPkT;
  const int64_t ns = (nt - I + strip - 1) / strip;
  const int64_t nterm = ns + I;  // strip partials, then column partials of tiles (P, I), P < I
  double s0 = 0.0, s1 = 0.0;
  int64_t k = h;
  for (; k + kRedSplit < nterm; k += 2 * kRedSplit) {
    const double a = k < ns ? rowpart[(size_t(I) * nsx + k) * kPkT + r]
                            : colpart[size_t(pk_tile_index(k - ns, I, nt)) * kPkT + r];
    const int64_t k2 = k + kRedSplit;
    const double b = k2 < ns ? rowpart[(size_t(I) * nsx + k2) * kPkT + r]
                             : colpart[size_t(pk_tile_index(k2 - ns, I, nt)) * kPkT + r];
    s0 += a;
    s1 += b;
  }
  if (k < nterm)
    s0 += k < ns ? rowpart[(size_t(I) * nsx + k) * kPkT + r] : colpart[size_t(pk_tile_index(k - ns, I, nt)) * kPkT + r];
  part[h][r] = s0 + s1;
  __syncthreads();
  const int64_t i = I * kPkT + r;
  if (h == 0 && i < n) {
    double t = part[0][r];
#pragma unroll
    for (int q = 1; q < kRedSplit; ++q) t += part[q][r];
    u[i * ldu] = t;
  }
}

size_t kapply_scratch_doubles(const KMat& km, int64_t n) {
  // row layout: up to 64 column segments; packed: strip 1 has the most partials
  return km.layout == 1 ? packed_scratch_doubles(n, 1) : size_t(64) * size_t(n);
}

size_t packed_scratch_doubles(int64_t n, int strip) {
  const int64_t nt = (n + kPkT - 1) / kPkT;
  const int64_t nsx = (nt + strip - 1) / strip;
  return size_t(nt) * nsx * kPkT + size_t(packed_tile_count(n)) * kPkT;
}

// Map 4 keeps nt x nb row partials and nb x nt column partials (nb = blocks
// per side); for B >= 2 that is within the strip-1 figure above.
size_t packed_shape_scratch_doubles(int64_t n, const PackedShape& s) {
  if (s.map != 4 && s.map != 5) return packed_scratch_doubles(n, s.strip);
  const int64_t nt = (n + kPkT - 1) / kPkT;
  const int64_t nb = (nt + s.strip - 1) / s.strip;
  return 2 * size_t(nt) * nb * kPkT;
}

namespace {
std::mutex g_pk_mu;
PackedShape g_pk_shape[2][2];  // [bf16][exact]
bool g_pk_set[2][2] = {};

template <bool BF16, bool EXACT>
void packed_launch(int map, dim3 grid, const void* K, int64_t n, int64_t nt, int strip, int64_t nsx, const float* v32,
                   const double* v64, double* rowpart, double* colpart, hipStream_t st) {
  // maps 2 and 3 with BF16 entries and FP64 sums would stage 66 KB of column
  // sums in LDS; they run as map 0
  const int64_t nstrips = grid.x;
  if constexpr (!(BF16 && EXACT)) {
    if (map == 2 || map == 3) {
      // map 3: persistent, four workgroups per CU walk the strips
      const dim3 g(map == 3 ? unsigned(std::min<int64_t>(nstrips, 1024)) : grid.x);
      kapply_packed_rows_kernel<BF16, EXACT, 512><<<g, 512, 0, st>>>(K, n, nt, strip, nsx, v32, v64, rowpart, colpart,
                                                                      nstrips);
      return;
    }
  }
  if (map == 1)
    kapply_packed_cols_kernel<BF16, EXACT><<<grid, 256, 0, st>>>(K, n, nt, strip, nsx, v32, v64, rowpart, colpart);
  else
    kapply_packed_rows_kernel<BF16, EXACT, 256><<<grid, 256, 0, st>>>(K, n, nt, strip, nsx, v32, v64, rowpart,
                                                                       colpart, nstrips);
}
template <int B, bool WIDE>
void packed_blocks_launch(bool bf, bool exact, dim3 grid, const void* K, int64_t n, int64_t nt, int64_t nb,
                          const float* v32, const double* v64, double* rowpart, double* colpart, hipStream_t st) {
  if (bf && exact)
    kapply_packed_blocks_kernel<true, true, B, WIDE><<<grid, 256, 0, st>>>(K, n, nt, nb, v32, v64, rowpart, colpart);
  else if (bf)
    kapply_packed_blocks_kernel<true, false, B, WIDE><<<grid, 256, 0, st>>>(K, n, nt, nb, v32, v64, rowpart, colpart);
  else if (exact)
    kapply_packed_blocks_kernel<false, true, B, WIDE><<<grid, 256, 0, st>>>(K, n, nt, nb, v32, v64, rowpart, colpart);
  else
    kapply_packed_blocks_kernel<false, false, B, WIDE><<<grid, 256, 0, st>>>(K, n, nt, nb, v32, v64, rowpart,
                                                                             colpart);
}
}  // namespace

PackedShape default_packed_shape(int dtype, int exact) {
  std::lock_guard<std::mutex> lk(g_pk_mu);
  const int d = dtype == KQR_BF16, e = exact != 0;
  if (g_pk_set[d][e]) return g_pk_shape[d][e];
  // fastest when swept at n = 50,000 (with the reduction; a later shape only
  // when 2 % faster): FP32 fast map 4, blocks of 4 x 4 tiles (820 us; map 5
  // 817 us), FP32 exact and BF16 fast map 5, blocks of 4 x 4 tiles (817 and
  // 445 us), BF16 exact map 0 / strip 16 (532 us)
  if (d) return e ? PackedShape{0, 16} : PackedShape{5, 4};
  return e ? PackedShape{5, 4} : PackedShape{4, 4};
}

void set_packed_shape(int dtype, int exact, PackedShape s) {
  std::lock_guard<std::mutex> lk(g_pk_mu);
  const int d = dtype == KQR_BF16, e = exact != 0;
  g_pk_shape[d][e] = s;
  g_pk_set[d][e] = true;
}

bool packed_shape_supported(const PackedShape& s) {
  if (s.map == 4 || s.map == 5) return s.strip == 2 || s.strip == 4;  // blocks of strip x strip tiles
  return s.map >= 0 && s.map <= 3 && s.strip >= 1 && s.strip <= kPkMaxStrip;
}

void kapply_packed(const KMat& km, int64_t n, const float* v32, const double* v64, double* u, int64_t ldu,
                   bool exact, hipStream_t st, const PackedShape* shape, double* scratch) {
  if (n <= 0) return;
  const PackedShape sh = shape ? *shape : default_packed_shape(km.dtype, exact);
  if (!packed_shape_supported(sh)) fail(KQR_EINVAL, "unsupported packed shape map=%d strip=%d", sh.map, sh.strip);
  const int strip = sh.strip;
  const int64_t nt = (n + kPkT - 1) / kPkT;
  const int64_t nsx = (nt + strip - 1) / strip;
  const size_t need = packed_shape_scratch_doubles(n, sh);
  double* buf = scratch;
  if (!buf) KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&buf), need * sizeof(double), st));
  const bool bf = km.dtype == KQR_BF16;
  if (sh.map == 4 || sh.map == 5) {
    const int64_t nb = (nt + strip - 1) / strip;
    double* rowpart = buf;
    double* colpart = buf + size_t(nt) * nb * kPkT;
    const dim3 grid((unsigned)(nb * (nb + 1) / 2));
    const bool wide = sh.map == 5;
    if (strip == 2 && wide) packed_blocks_launch<2, true>(bf, exact, grid, km.K, n, nt, nb, v32, v64, rowpart, colpart, st);
    else if (strip == 2) packed_blocks_launch<2, false>(bf, exact, grid, km.K, n, nt, nb, v32, v64, rowpart, colpart, st);
    else if (wide) packed_blocks_launch<4, true>(bf, exact, grid, km.K, n, nt, nb, v32, v64, rowpart, colpart, st);
    else packed_blocks_launch<4, false>(bf, exact, grid, km.K, n, nt, nb, v32, v64, rowpart, colpart, st);
    KQR_LAUNCH_CHECK();
    packed_reduce_blocks_kernel<<<dim3((unsigned)nt), kPkT * 4, 0, st>>>(rowpart, colpart, n, nt, nb, strip, u, ldu);
    KQR_LAUNCH_CHECK();
    if (!scratch) KQR_CHECK_HIP(hipFreeAsync(buf, st));
    return;
  }
  double* rowpart = buf;
  double* colpart = buf + size_t(nt) * nsx * kPkT;
  const dim3 grid((unsigned)pk_strips_tail(nt, strip));  // exactly the strips (no idle workgroups)
  if (exact && bf) packed_launch<true, true>(sh.map, grid, km.K, n, nt, strip, nsx, v32, v64, rowpart, colpart, st);
  else if (exact) packed_launch<false, true>(sh.map, grid, km.K, n, nt, strip, nsx, v32, v64, rowpart, colpart, st);
  else if (bf) packed_launch<true, false>(sh.map, grid, km.K, n, nt, strip, nsx, v32, v64, rowpart, colpart, st);
  else packed_launch<false, false>(sh.map, grid, km.K, n, nt, strip, nsx, v32, v64, rowpart, colpart, st);
  KQR_LAUNCH_CHECK();
  packed_reduce(rowpart, colpart, n, strip, u, ldu, st);
  if (!scratch) KQR_CHECK_HIP(hipFreeAsync(buf, st));
}

void packed_reduce(const double* rowpart, const double* colpart, int64_t n, int strip, double* u, int64_t ldu,
                   hipStream_t st) {
  const int64_t nt = (n + kPkT - 1) / kPkT;
  const int64_t nsx = (nt + strip - 1) / strip;
  packed_reduce_kernel<<<dim3((unsigned)nt), kPkT * kRedSplit, 0, st>>>(rowpart, colpart, n, nt, strip, nsx, u, ldu);
  KQR_LAUNCH_CHECK();
}

// ================================================================= one row
template <bool BF16>
__global__ void krow_from_packed_kernel(const void* __restrict__ K, int64_t n, int64_t nt, int64_t s,
                                        double* __restrict__ out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const size_t off = pk_offset(s, j, nt);  // K[s][j], or K[j][s] below the diagonal tiles
  if (BF16) out[j] = __uint_as_float(uint32_t(static_cast<const uint16_t*>(K)[off]) << 16);
  else out[j] = static_cast<const float*>(K)[off];
}

void kernel_row_packed(const KMat& km, int64_t n, int64_t s, double* out, hipStream_t st) {
  const int64_t nt = (n + kPkT - 1) / kPkT;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (km.dtype == KQR_BF16) krow_from_packed_kernel<true><<<grid, 256, 0, st>>>(km.K, n, nt, s, out);
  else krow_from_packed_kernel<false><<<grid, 256, 0, st>>>(km.K, n, nt, s, out);
  KQR_LAUNCH_CHECK();
}

}  // namespace kqr
