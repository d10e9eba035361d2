// Products with constant matrices on the gfx950 matrix cores, for the
// DCT-as-GEMM variant of the step: both operands split into three bfloat16
// parts (x = x_0 + x_1 + x_2 + O(2^-25 |x|)), and the six products of parts
// whose orders add up to at most 2 accumulated in FP32 by
// v_mfma_f32_32x32x16_bf16 -- the rounding of an FP32 product (the three
// terms left out are below 2^-26 of the result's terms).
//
// Every product of the step pairs a constant matrix d (a DCT matrix, its
// transpose, or a DFT matrix of the factored transforms, split once at
// context creation, row-major with K contiguous) with an FP32 data operand x
// that is split while it is staged into LDS, so no separate splitting pass
// touches HBM:
//   row mode (transforms along x): C(m, n) = sum_k d[m K + k] x[n ldx + k],
//     the data rows of all fields stacked along n;
//   column mode (transforms along y): C(m, n) = sum_k x[k ldx + m] d[n K + k],
//     one field (or block of a field) per batch entry.
// Both write C(m, n) at c[n ldc + m], so that an output row is contiguous,
// or pass it through an epilogue of the factored transforms
// (gemm_fourstep.hpp).
#pragma once
#include <stdint.h>

#include "gemm_dct.hpp"
#include "gemm_fourstep.hpp"

namespace ccm {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));

enum MfMode { MF_ROW = 0, MF_COL = 1 };

constexpr int MF_THREADS = 256;   // four waves, each owning a quarter of the block tile
constexpr int MF_BK = 32;         // K per staged slice
// LDS line of one tile line: 32 bf16 of K (four 16-byte chunks, 64 bytes).
constexpr int MF_ROW16 = 4;       // 16-byte units per LDS line

// Tile edge along m and n: 128, or 64 for the smallest grids.
__host__ __device__ constexpr int mf_tile(int dim) { return dim >= 128 ? 128 : 64; }

// LDS slot of K chunk k8 of a line: the chunks of line l are permuted by
// k8 ^ ((l >> 2) & 3). The 256-byte bank window holds 16 chunks; 16
// consecutive lanes then hit 16 distinct bank groups both when four lanes
// stage the four chunks of one line (4 lines per 16 lanes, one (l >> 2)) and
// when 16 lanes read one chunk of 16 consecutive lines (fragment loads).
__device__ __forceinline__ int mf_slot(int line, int k8) {
  return line * MF_ROW16 + (k8 ^ ((line >> 2) & 3));
}

// bf16 parts of each operand.
constexpr int MF_PARTS = 3;

// x = x_0 + x_1 + x_2 + O(2^-25 |x|): three bfloat16 parts of eight FP32
// values, each the rounding of what the earlier parts leave.
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8_t (&part)[MF_PARTS]) {
  float r[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = v[e];
#pragma unroll
  for (int q = 0; q < MF_PARTS; ++q) {
    u16x8_t h;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      h[e] = bf16_rne(r[e]);
      r[e] -= bf16_to_f32(h[e]);
    }
    part[q] = __builtin_bit_cast(bf16x8_t, h);
  }
}

// A constant matrix operand as its bf16 parts (hi, mid, lo), each row-major
// with K contiguous.
struct MfMat {
  const uint16_t* part[MF_PARTS];
};

// Block tile (m0, n0) and batch entry z of block b: blocks are spread over
// the eight XCDs in contiguous ranges (xcd_remap), and within a batch entry
// the tiles go in groups of 8 x 8, so that the blocks one XCD holds at once
// share eight m-slices and eight n-slices of the operands in its L2.
__device__ __forceinline__ void mf_block_tile(int mb_count, int nb_count, int& z, int& mb,
                                              int& nb) {
  const int total = gridDim.x;
  const int b = xcd_remap(blockIdx.x, total);
  const int per = mb_count * nb_count;
  z = b / per;
  const int t = b - z * per;
  if ((mb_count & 7) == 0 && (nb_count & 7) == 0) {
    const int g = t >> 6, w = t & 63;
    const int gm = mb_count >> 3;
    mb = (g % gm) * 8 + (w & 7);
    nb = (g / gm) * 8 + (w >> 3);
  } else {
    mb = t % mb_count;
    nb = t / mb_count;
  }
}

// C = the product of MODE (above) for an M x N tile grid of BM x BN blocks,
// batch entries z = 0 .. gridDim.x / (M/BM N/BN) - 1 at strides sx (x) and sc
// (c); d is shared by the batch. EPI: how C is stored (FsEpilogue); XL: how
// the data operand is read (FsLoad, column mode).
template <int MODE, int BM, int BN, int EPI, int XL>
__global__ void __launch_bounds__(MF_THREADS)
k_gemm_bf16x3(MfMat d, const float* __restrict__ x, float* __restrict__ c, int M, int N, int K,
              int ldx, int ldc, size_t sx, size_t sc, FsArgs fa) {
  constexpr bool SWAP = fs_swapped(EPI);
  constexpr int PT = MF_PARTS;
  static_assert(XL == XL_PLAIN || MODE == MF_COL, "the fused loads are column-mode operands");
  constexpr int TM = BM / 64, TN = BN / 64;   // 32 x 32 subtiles per wave along m, n
  // LDS tiles per part: lines indexed by m (Lm) and by n (Ln), K contiguous.
  __shared__ bf16x8_t Lm[PT][BM * MF_ROW16];
  __shared__ bf16x8_t Ln[PT][BN * MF_ROW16];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int z, mb, nb;
  mf_block_tile(M / BM, N / BN, z, mb, nb);
  const int m0 = mb * BM, n0 = nb * BN;
  const float* xz = x + (size_t)z * sx;
  float* cz = c + (size_t)z * sc;

  // Staging: the d tile is (rows R0 .., K slice) with R = m (row mode) or n
  // (column mode); the x tile is (rows S0 .., K slice) with S the other one.
  constexpr int RD = MODE == MF_ROW ? BM : BN;   // lines of the d tile
  constexpr int RX = MODE == MF_ROW ? BN : BM;   // lines of the x tile
  constexpr int CD = RD * 4 / MF_THREADS;        // 16-byte chunks per thread (d)
  constexpr int CX = RX * 4 / MF_THREADS;        // 8-value chunks per thread (x)
  const int d0 = MODE == MF_ROW ? m0 : n0;
  const int x0 = MODE == MF_ROW ? n0 : m0;
  // LDS slot i of part q of the d tile and of the x tile
  auto ld = [&](int q, int i) -> bf16x8_t& {
    if constexpr (MODE == MF_ROW) return Lm[q][i]; else return Ln[q][i];
  };
  auto lx = [&](int q, int i) -> bf16x8_t& {
    if constexpr (MODE == MF_ROW) return Ln[q][i]; else return Lm[q][i];
  };

  bf16x8_t rd[CD][PT];
  float rx[CX][8];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < CD; ++i) {
      // four consecutive lanes read the 64 contiguous bytes of one line
      const int ch = tid + i * MF_THREADS;
      const int r = ch >> 2, k8 = ch & 3;
      const size_t o = (size_t)(d0 + r) * K + k0 + 8 * k8;
#pragma unroll
      for (int q = 0; q < PT; ++q) rd[i][q] = *reinterpret_cast<const bf16x8_t*>(d.part[q] + o);
    }
#pragma unroll
    for (int i = 0; i < CX; ++i) {
      const int ch = tid + i * MF_THREADS;
      if constexpr (MODE == MF_ROW) {
        // line s = n, eight consecutive k of a data row (two 16-byte loads)
        const int s = ch >> 2, k8 = ch & 3;
        const f32x4_t* p =
            reinterpret_cast<const f32x4_t*>(xz + (size_t)(x0 + s) * ldx + k0 + 8 * k8);
        const f32x4_t a = p[0], b = p[1];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          rx[i][e] = a[e];
          rx[i][4 + e] = b[e];
        }
      } else {
        // line s = m, eight consecutive k: consecutive lanes read consecutive m
        const int s = ch % RX, k8 = ch / RX;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if constexpr (XL == XL_PLAIN)
            rx[i][e] = xz[(size_t)(k0 + 8 * k8 + e) * ldx + x0 + s];
          else
            rx[i][e] = fs_load<XL>(x, (uint32_t)z, (uint32_t)(k0 + 8 * k8 + e), (uint32_t)(x0 + s), fa);
        }
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int i = 0; i < CD; ++i) {
      const int ch = tid + i * MF_THREADS;
      const int r = ch >> 2, k8 = ch & 3;
#pragma unroll
      for (int q = 0; q < PT; ++q) ld(q, mf_slot(r, k8)) = rd[i][q];
    }
#pragma unroll
    for (int i = 0; i < CX; ++i) {
      const int ch = tid + i * MF_THREADS;
      // row mode: four lanes per line; column mode: consecutive lanes, consecutive lines
      const int s = MODE == MF_ROW ? ch >> 2 : ch % RX;
      const int k8 = MODE == MF_ROW ? ch & 3 : ch / RX;
      bf16x8_t part[PT];
      split8(rx[i], part);
#pragma unroll
      for (int q = 0; q < PT; ++q) lx(q, mf_slot(s, k8)) = part[q];
    }
  };

  // Wave tile: n range wn .. wn + BN/2, m range wm .. wm + BM/2.
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
  f32x16_t acc[TN][TM];
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;

  // ac += (n-line fragment an) x (m-line fragment bm), operands in the
  // order the accumulator layout asks for.
  auto mma = [&](f32x16_t& ac, const bf16x8_t& an, const bf16x8_t& bm) {
    ac = SWAP ? __builtin_amdgcn_mfma_f32_32x32x16_bf16(bm, an, ac, 0, 0, 0)
              : __builtin_amdgcn_mfma_f32_32x32x16_bf16(an, bm, ac, 0, 0, 0);
  };

  fetch(0);
  for (int k0 = 0; k0 < K; k0 += MF_BK) {
    __syncthreads();                 // the previous slice's fragments are read
    stage();
    __syncthreads();
    if (k0 + MF_BK < K) fetch(k0 + MF_BK);   // next slice in flight during the products
#pragma unroll
    for (int ks = 0; ks < MF_BK / 16; ++ks) {
      const int kc = ks * 2 + (lane >> 5);  // this lane's 8 k of the 16
      bf16x8_t an[PT][TN], bm[PT][TM];
#pragma unroll
      for (int q = 0; q < PT; ++q) {
#pragma unroll
        for (int a = 0; a < TN; ++a) an[q][a] = Ln[q][mf_slot(wn + a * 32 + (lane & 31), kc)];
#pragma unroll
        for (int b = 0; b < TM; ++b) bm[q][b] = Lm[q][mf_slot(wm + b * 32 + (lane & 31), kc)];
      }
#pragma unroll
      for (int a = 0; a < TN; ++a)
#pragma unroll
        for (int b = 0; b < TM; ++b) {
          // the smaller terms first
          mma(acc[a][b], an[1][a], bm[1][b]);
          mma(acc[a][b], an[0][a], bm[2][b]);
          mma(acc[a][b], an[2][a], bm[0][b]);
          mma(acc[a][b], an[0][a], bm[1][b]);
          mma(acc[a][b], an[1][a], bm[0][b]);
          mma(acc[a][b], an[0][a], bm[0][b]);
        }
    }
  }
  // Accumulator element v of lane l: MFMA row (v/4) 8 + (l/32) 4 + v%4, column
  // l % 32; rows are n and columns m (swapped: the other way round). Elements
  // v and v + 1 (v even) are two consecutive rows of one column.
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      const int mb0 = m0 + wm + b * 32, nb0 = n0 + wn + a * 32;
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        const int r = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        const int m = SWAP ? mb0 + r : mb0 + (lane & 31);
        const int n = SWAP ? nb0 + (lane & 31) : nb0 + r;
        if constexpr (EPI == EPI_STORE) {
          cz[(size_t)n * ldc + m] = acc[a][b][v];
          cz[(size_t)(n + 1) * ldc + m] = acc[a][b][v + 1];
        } else {
          fs_epilogue<EPI>(cz, ldc, (uint32_t)z, (uint32_t)m, (uint32_t)n, acc[a][b][v],
                           acc[a][b][v + 1], fa);
        }
      }
    }
}

}  // namespace ccm
