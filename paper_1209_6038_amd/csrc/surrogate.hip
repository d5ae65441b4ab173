// surrogate.hip -- multilayer-perceptron surrogate of the cloak transit:
// entry ray on the outer cylinder -> exit ray and optical path length.
//
// Network: 6 inputs -> 256 -> 256 -> 256 -> 256 -> 5 outputs, SiLU after the
// four hidden layers; inputs and targets are standardized with offsets and
// scales stored in the model. Precision by layer:
//   layer 1 (6 -> 256) and layer 5 (256 -> 5): FP32 on the vector units
//     (too thin for matrix cores; FP32 keeps the inputs' and outputs'
//     precision),
//   layers 2-4 (256 -> 256, 98% of the flops): BF16 x BF16 products with
//     FP32 accumulation on MFMA (v_mfma_f32_16x16x32_bf16).
// Training minimizes the mean squared error of the standardized targets
// with AdamW on FP32 master weights; the BF16 copies of W2..W4 are refreshed
// after every step.
//
// The surrogate is not part of the paper. The exact integrator
// (rt_transit_exact) labels its training data, judges its error, and
// replaces its prediction wherever the gate rejects it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/rt.h"
#include "internal.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace sg {

constexpr int NIN = 6, HID = 256, NOUT = 5;
// FP32 parameter vector, weights stored (fan_in, fan_out) row-major:
// W1 [6][256], b1, W2 [256][256], b2, W3, b3, W4, b4, W5 [256][5], b5 [5]
constexpr long long OFF_W1 = 0;
constexpr long long OFF_B1 = OFF_W1 + NIN * HID;
constexpr long long OFF_W2 = OFF_B1 + HID;
constexpr long long OFF_B2 = OFF_W2 + HID * HID;
constexpr long long OFF_W3 = OFF_B2 + HID;
constexpr long long OFF_B3 = OFF_W3 + HID * HID;
constexpr long long OFF_W4 = OFF_B3 + HID;
constexpr long long OFF_B4 = OFF_W4 + HID * HID;
constexpr long long OFF_W5 = OFF_B4 + HID;
constexpr long long OFF_B5 = OFF_W5 + HID * NOUT;
constexpr long long NPARAM = OFF_B5 + NOUT;  // 200,453
static_assert(OFF_B1 == OFF_W1 + NIN * HID, "W1, b1 are contiguous");
// BF16 copies of W2, W3, W4: transposed [out][in] (forward: the 8
// consecutive inputs an MFMA lane needs for one output are one 16-byte
// load) and row-major [in][out] (backward through the layer); NBF per copy
constexpr long long NBF = 3LL * HID * HID;
// scaling block: in_off[6], in_scale[6], out_mean[5], out_std[5], then the loss
constexpr int S_INOFF = 0, S_INSCALE = 6, S_OMEAN = 12, S_OSTD = 17, S_LOSS = 22, NSCAL = 24;
// trust map of the side job: (axis, branch) x alpha cells x beta cells
constexpr int NCELL_A = 128, NCELL_B = 128, NCOMBO = 4;
constexpr int NCELLS = NCOMBO * NCELL_A * NCELL_B;
// trust map of the cap job: (axis, branch) x alpha x |beta| x cap-fraction
// cells, as many as the side job's
constexpr int CAP_A = 32, CAP_B = 16, CAP_U = 32;
static_assert(NCOMBO * CAP_A * CAP_B * CAP_U == NCELLS, "both jobs' trust maps have NCELLS cells");
constexpr float OUT_STD_FLOOR = 1e-3f;
constexpr float PI_F = 3.14159265358979f;

}  // namespace sg

// the library's thread-local error message (shared with the tracer)
void rt_set_error_message(const char *msg);

namespace sg {

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  rt_set_error_message(buf);
  return code;
}

// SiLU and its derivative with the hardware reciprocal (about 1 ulp): the
// activations are rounded to BF16 or feed FP32 layers whose inputs carry
// far more error than that, and an IEEE division would cost ~10
// instructions per activation. Training and inference share these.
__device__ __forceinline__ float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_f(float z) { return z * sigmoid_f(z); }
__device__ __forceinline__ float dsilu_f(float z) {
  const float s = sigmoid_f(z);
  return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// Tiled GEMM on MFMA: C(M x N) = A(M x K) B(K x N) with both operands
// contiguous along K (A(i,k) = A[i*lda + k], B(k,j) = B[j*ldb + k]), BF16 in, FP32
// accumulation. 64 x 64 tile per 256-thread block (4 waves of 32 x 32, each
// 2 x 2 MFMA 16x16x32 tiles), K in steps of 32 staged through LDS, optionally
// split over K (each split covers `kchunk` of K). One-dimensional grid of
// (column tiles) x (row tiles) x (splits) blocks, the column tile fastest.
// Consecutive blocks go to the 8 XCDs in turn, each with its own L2, so the
// block number is first renumbered to give each XCD a contiguous range of
// tiles: the column tiles of a row tile (which read the same A rows), and the
// tiles of a K split (which read the same A and B columns), then share an L2.
// Epilogues (the backward pass of the BF16 layers):
//   EPI_DSILU      g = acc * silu'(Z): Cf <- g, Cb <- bf16(g), its
//                  transpose Cbt <- bf16(g)^T ([N][ldcbt]), and the
//                  block's column sums of g to the row of colsum of its
//                  row tile (a partial-sum array [row tiles][N], may be NULL;
//                  with xf, [row tiles][7][N] holding xf^T g, then the sums:
//                  the gradients of W1 and b1 when g is dz of layer 1)
//   EPI_SPLIT      Cf + split * M * ldcf <- acc: one partial product per K
//                  split, summed afterwards by k_sum_rows
// (each output pointer may be NULL)
// ---------------------------------------------------------------------------
enum { EPI_DSILU = 1, EPI_SPLIT = 2 };

struct Gemm {
  const bf16 *A;
  long long lda;  // A(i, k) = A[i * lda + k]
  const bf16 *B;
  long long ldb;  // B(k, j) = B[j * ldb + k]
  bool veca, vecb;  // 16-byte operand loads allowed
  int M, N, K, kchunk, epi;
  int nct, nrt;  // column and row tiles
  const float *Z;
  long long ldz;
  float *Cf;
  long long ldcf;
  bf16 *Cb;
  long long ldcb;
  float *colsum;  // EPI_DSILU: per-block column sums of g, [row tile][N] (may be NULL)
  const float *xf;  // with colsum: the layer-1 inputs [M][6], for the sums xf^T g ([row tile][7][N])
  bf16 *Cbt;      // EPI_DSILU: bf16(g) transposed, Cbt[col * ldcbt + row] (may be NULL)
  long long ldcbt;
};

// Operand tiles are staged 64 deep in K: a 64 x 64 BF16 tile (rows r0..,
// k k0..) is two 16-byte vectors per thread, 8 consecutive threads on the 128
// bytes of one row. P(row, k) = P[row * ld + k] (K contiguous); rows < nrow
// and k < kend valid, zeros elsewhere (vec: ld and P allow 16-byte loads).
constexpr int GT = 64, GK = 64, GLD = GK + 8;  // tile, K step, padded LDS row

__device__ __forceinline__ void load_op(bf16x8 v[2], const bf16 *__restrict__ P, long long ld, bool vec, int r0,
                                        int nrow, int k0, int kend, int tid) {
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int gr = r0 + (tid >> 3) + 32 * p, gk = k0 + 8 * (tid & 7);
    const bf16 *src = P + (long long)gr * ld + gk;
    if (vec && gr < nrow && gk + 8 <= kend) {
      v[p] = *reinterpret_cast<const bf16x8 *>(src);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[p][e] = (gr < nrow && gk + e < kend) ? src[e] : (bf16)0.0f;
    }
  }
}

__device__ __forceinline__ void store_op(bf16 *T, const bf16x8 v[2], int tid) {
#pragma unroll
  for (int p = 0; p < 2; ++p) *reinterpret_cast<bf16x8 *>(&T[((tid >> 3) + 32 * p) * GLD + 8 * (tid & 7)]) = v[p];
}

// C = A B over the block's K range with an epilogue: a 64 x 64 tile, 4 waves
// in 2 x 2, each owning 32 x 32 outputs as 2 x 2 MFMA 16x16x32 tiles. The K
// loop is double-buffered: step i's tiles go from registers to one LDS stage
// while step i + 1's global loads are in flight, so one barrier per 64-deep
// step; the epilogue's inputs (the pre-activations) are loaded before the
// loop. The FP32 output tile reuses the staging area.
__global__ void __launch_bounds__(256) k_gemm(Gemm g) {
  constexpr int BM = GT, BN = GT, WM = 2, WN = 2, STAGE = (BM + BN) * GLD;
  __shared__ __attribute__((aligned(16))) bf16 sm[2 * STAGE];
  static_assert(BM * (BN + 4) * sizeof(float) <= sizeof(sm), "the FP32 tile fits in the staging area");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned t = (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);  // a bijection of [0, nb)
  const int ct = (int)(t % (unsigned)g.nct), rt = (int)(t / (unsigned)g.nct % (unsigned)g.nrt);
  const int split = (int)(t / (unsigned)g.nct / (unsigned)g.nrt);
  const int row0 = rt * BM, col0 = ct * BN;
  const int kbeg = split * g.kchunk, kend = min(g.K, kbeg + g.kchunk);
  // this thread's 16 epilogue entries: row lr, columns lc.. of the tile
  const int lr = tid >> 2, lc = (tid & 3) * 16;
  float zp[16];
  const bool zpre = g.epi == EPI_DSILU && row0 + lr < g.M && col0 + lc + 16 <= g.N;
  if (zpre) {
    const float *zr = g.Z + (long long)(row0 + lr) * g.ldz + col0 + lc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 zz = *reinterpret_cast<const float4 *>(zr + 4 * q);
      zp[4 * q] = zz.x; zp[4 * q + 1] = zz.y; zp[4 * q + 2] = zz.z; zp[4 * q + 3] = zz.w;
    }
  }
  f32x4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // A(i, k) = A[i*lda + k]; B staged as its transpose, B(k, j) = B[j*ldb + k]
  bf16x8 ra[2], rb[2];
  load_op(ra, g.A, g.lda, g.veca, row0, g.M, kbeg, kend, tid);
  load_op(rb, g.B, g.ldb, g.vecb, col0, g.N, kbeg, kend, tid);
  const int nk = (kend - kbeg + GK - 1) / GK;
  for (int it = 0; it < nk; ++it) {
    bf16 *As = sm + (it & 1) * STAGE, *Bs = As + BM * GLD;
    store_op(As, ra, tid);
    store_op(Bs, rb, tid);
    __syncthreads();  // also: every wave is done with this stage's previous use (step it - 2)
    if (it + 1 < nk) {
      const int k1 = kbeg + (it + 1) * GK;
      load_op(ra, g.A, g.lda, g.veca, row0, g.M, k1, kend, tid);
      load_op(rb, g.B, g.ldb, g.vecb, col0, g.N, k1, kend, tid);
    }
    // operand layout of v_mfma_f32_16x16x32_bf16: lane l holds
    // A[l%16][8*(l/16) + j] and B[8*(l/16) + j][l%16], j = 0..7 (padded rows
    // of 144 bytes keep each 8-element read 16-byte aligned and spread the
    // 16 rows of a read over all banks)
#pragma unroll
    for (int ks = 0; ks < GK; ks += 32) {
      bf16x8 af[WM], bfr[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i)
        af[i] = *reinterpret_cast<const bf16x8 *>(&As[(wm * 32 + i * 16 + (lane & 15)) * GLD + ks + 8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < WN; ++j)
        bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[(wn * 32 + j * 16 + (lane & 15)) * GLD + ks + 8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave has read its last operands: the staging area becomes the FP32 tile
  // result layout: lane l holds D[4*(l/16) + i][l%16], i = 0..3
  // the elementwise epilogues read and write whole rows: the tile goes
  // through LDS, and each thread then owns 16 consecutive columns of a row
  // (64-byte FP32 and 32-byte BF16 vectors, full cache lines per row)
  float(*Cs)[BN + 4] = reinterpret_cast<float(*)[BN + 4]>(sm);
  // beyond the FP32 tile: the layer-1 inputs of the tile's rows [64][6] and
  // the column sums of the 4 waves [4][7][64]
  float *const xs = &Cs[BM][0];
  float *const red = xs + BM * NIN;
  static_assert((BM * (BN + 4) + BM * NIN + 4 * (NIN + 1) * 64) * sizeof(float) <= sizeof(sm), "epilogue LDS");
  if (g.epi == EPI_DSILU && g.colsum && g.xf)
    for (int e = tid; e < BM * NIN; e += 256) {
      const int r = e / NIN;
      xs[e] = row0 + r < g.M ? g.xf[(long long)(row0 + r) * NIN + e % NIN] : 0.0f;
    }
#pragma unroll
  for (int ti = 0; ti < WM; ++ti)
#pragma unroll
    for (int tj = 0; tj < WN; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Cs[wm * 16 * WM + ti * 16 + 4 * (lane >> 4) + r][wn * 16 * WN + tj * 16 + (lane & 15)] = acc[ti][tj][r];
  __syncthreads();
  static_assert(BM == 64 && BN == 64, "one epilogue pass: 16 entries per thread");
  do {
    const int row = row0 + lr, col = col0 + lc;
    const bool sums = g.epi == EPI_DSILU && (g.colsum || g.Cbt);  // g stays in the tile
    if (row >= g.M) {
      if (sums) {
#pragma unroll
        for (int e = 0; e < 16; ++e) Cs[lr][lc + e] = 0.0f;
      }
      break;
    }
    float v[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = *reinterpret_cast<const float4 *>(&Cs[lr][lc + 4 * q]);
      v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
    }
    if (g.epi == EPI_SPLIT) {
      float *o = g.Cf + (long long)split * g.M * g.ldcf + (long long)row * g.ldcf + col;
      if (col + 16 <= g.N) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *reinterpret_cast<float4 *>(o + 4 * q) = float4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
      } else {
        for (int e = 0; e < 16 && col + e < g.N; ++e) o[e] = v[e];
      }
      break;
    }
    if (col + 16 <= g.N) {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] *= dsilu_f(zp[e]);  // zpre holds here
      if (g.Cf) {
        float *o = g.Cf + (long long)row * g.ldcf + col;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *reinterpret_cast<float4 *>(o + 4 * q) = float4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
      }
      if (g.Cb) {
        bf16x8 b0, b1;
#pragma unroll
        for (int e = 0; e < 8; ++e) { b0[e] = (bf16)v[e]; b1[e] = (bf16)v[8 + e]; }
        bf16 *o = g.Cb + (long long)row * g.ldcb + col;
        *reinterpret_cast<bf16x8 *>(o) = b0;
        *reinterpret_cast<bf16x8 *>(o + 8) = b1;
      }
      if (sums) {
        // this thread's own 16 entries of the staged tile, now holding g
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *reinterpret_cast<float4 *>(&Cs[lr][lc + 4 * q]) = float4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
      }
    } else {
      for (int e = 0; e < 16; ++e) {
        const long long c = col + e;
        const float d = c < g.N ? v[e] * dsilu_f(g.Z[row * g.ldz + c]) : 0.0f;
        if (sums) Cs[lr][lc + e] = d;
        if (c >= g.N) continue;
        if (g.Cf) g.Cf[row * g.ldcf + c] = d;
        if (g.Cb) g.Cb[row * g.ldcb + c] = (bf16)d;
      }
    }
  } while (false);
  if (g.epi == EPI_DSILU && (g.colsum || g.Cbt)) __syncthreads();
  if (g.epi == EPI_DSILU && g.Cbt) {
    // every thread has left g (zeros outside the matrix) in its entries of
    // the staged tile: the transpose, 8 consecutive rows of one column per
    // 16-byte store
    // (BM / 8 consecutive threads on the consecutive pieces of one column)
    static_assert(BM % 8 == 0 && (BM / 8) * BN % 256 == 0, "transposed pieces per thread");
    for (int e = tid; e < (BM / 8) * BN; e += 256) {
      const int c = e / (BM / 8), r8 = (e % (BM / 8)) * 8;
      const int col = col0 + c, row = row0 + r8;
      if (col >= g.N || row >= g.M) continue;
      bf16 *o = g.Cbt + (long long)col * g.ldcbt + row;
      if (row + 8 <= g.M) {
        bf16x8 pk;
#pragma unroll
        for (int k = 0; k < 8; ++k) pk[k] = (bf16)Cs[r8 + k][c];
        *reinterpret_cast<bf16x8 *>(o) = pk;
      } else {
        for (int k = 0; row + k < g.M; ++k) o[k] = (bf16)Cs[r8 + k][c];
      }
    }
  }
  if (g.epi == EPI_DSILU && g.colsum) {
    // the tile's column sums of g and, with xf, before them the sums of
    // xf[row][k] g[row][col], k < 6: one row of partial sums per row tile,
    // [row tile][7][N] (or [row tile][N]), added up by k_sum_rows (no
    // atomics). Wave w sums rows 16 w .. 16 w + 15 for column `lane`, then
    // the 4 waves' sums are added through LDS.
    static_assert(BN == 64, "one column per lane");
    constexpr int NS = NIN + 1;
    float sk[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) sk[k] = 0.0f;
#pragma unroll 4
    for (int r = 16 * w; r < 16 * w + 16; ++r) {
      const float gv = Cs[r][lane];
      sk[NIN] += gv;
      if (g.xf) {
#pragma unroll
        for (int k = 0; k < NIN; ++k) sk[k] = fmaf(xs[r * NIN + k], gv, sk[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) red[(w * NS + k) * 64 + lane] = sk[k];
    __syncthreads();
    const int nsum = g.xf ? NS : 1;
    for (int e = tid; e < nsum * BN; e += 256) {
      const int k = e / BN, c = e % BN, src = g.xf ? k : NIN;
      const float v = (red[src * 64 + c] + red[(NS + src) * 64 + c]) +
                      (red[(2 * NS + src) * 64 + c] + red[(3 * NS + src) * 64 + c]);
      if (col0 + c < g.N) g.colsum[((long long)rt * nsum + k) * g.N + col0 + c] = v;
    }
  }
}

// dst[c] += sum over r < rows of part[r * ld + c], c < ncols. Block (x, y):
// 64 consecutive columns x 4 groups of rows y*4+q, y*4+q+4Y, ... (Y =
// gridDim.y) summed in registers, then over the 4 groups in LDS, one atomic
// per column and block row (gridDim.y = 1: a single writer per column).
__global__ void __launch_bounds__(256) k_sum_rows(const float *__restrict__ part, int rows, long long ld,
                                                  int ncols, float *__restrict__ dst) {
  __shared__ float sh[4][64];
  const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
  const long long col = (long long)blockIdx.x * 64 + c;
  float s0 = 0.f, s1 = 0.f;
  if (col < ncols) {
    const int step = 4 * gridDim.y;
    int r = blockIdx.y * 4 + q;
    for (; r + step < rows; r += 2 * step) {
      s0 += part[(long long)r * ld + col];
      s1 += part[(long long)(r + step) * ld + col];
    }
    if (r < rows) s0 += part[(long long)r * ld + col];
  }
  sh[q][c] = s0 + s1;
  __syncthreads();
  if (q == 0 && col < ncols) atomicAdd(&dst[col], (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]));
}

// ---------------------------------------------------------------------------
// Target encoding. Entry (phi, z, alpha, beta) on r = b, exit (phi', z',
// alpha', beta') on r = b, optical path T between them:
//   t0 = dtheta - dtheta_0,  t1 = dz - dz_0,  t2 = alpha' - alpha,
//   t3 = beta' - beta,       t4 = T - T_0,
// with dz = z' - z and dtheta the signed azimuth swept by the ray. The
// conserved angular momentum p_theta keeps its sign along the path (the
// inner mirror reflects radially), so theta is monotonic with the sign s of
// alpha, and dtheta = s * ((s (phi' - phi)) mod 2 pi) unwraps exactly for
// transits of less than a full turn. All five residuals are bounded: the
// refraction into the cloak keeps the rise and the path inside finite even
// for entries at grazing elevation, so they enter unscaled (a residual
// divided by cos(beta) would multiply the network's error by 1 / cos(beta)).
//
// (dtheta_0, dz_0, T_0) is the closed-form transit where one exists (zero
// otherwise), so that the network learns a residual:
//  - radial cloak, ordinary branch: M = kappa I (Eq. (14): eps_o = kappa),
//    a homogeneous medium of index n = sqrt(kappa) = b / (b - a); the ray is
//    straight inside, with horizontal wave number k_h = sqrt(n^2 - k_z^2)
//    and horizontal impact parameter p = b |k_theta| / k_h, and reflects
//    specularly off the metal cylinder when p <= a (Sect. 4);
//  - azimuthal cloak, extraordinary branch: M = diag(kappa, kappa s, kappa)
//    (Eq. (15)) makes the line element drho^2 + rho^2 dtheta^2 + dzeta^2 with
//    rho = sqrt(kappa) (r - a), zeta = sqrt(kappa) z: a straight line in
//    (rho, theta, zeta) at unit speed, entering at rho = b with tangential
//    speed k_theta and axial speed k_z / sqrt(kappa).
//  - radial cloak, extraordinary branch, and azimuthal cloak, ordinary
//    branch: both have m_theta = m_z = kappa s, so with p = b k_theta the
//    Hamiltonian constraint gives m_r rdot^2 = Q(r) / (kappa (r - a)^2) for
//    the quadratic Q(r) = kappa (r - a)^2 - p^2 - k_z^2 r^2, which equals
//    (b k_n)^2 at r = b; the turning point is its larger root. The sweep,
//    the rise and the optical path per unit r are
//      radial e (m_r = kappa):      p / (u sqrt Q), k_z r^2 / (u sqrt Q),
//                                   kappa u / sqrt Q            (u = r - a),
//      azimuthal o (m_r = kappa s): p / (r sqrt Q), k_z r / sqrt Q,
//                                   kappa u^2 / (r sqrt Q),
//    sums of 1 / sqrt Q, x / sqrt Q and 1 / (x sqrt Q) for Q quadratic in x,
//    integrated in closed form from the root to r = b (asinh, atan2 and
//    asinh(sqrt y) / sqrt y, the last continued through y = 0 as
//    asin(sqrt -y) / sqrt -y).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wrap2pi(float a) {
  a = fmodf(a, 2.0f * PI_F);
  return a < 0.0f ? a + 2.0f * PI_F : a;
}

// half the azimuth swept along a chord of a circle of radius 1 with impact
// parameter u in [0, 1]: acos(u), in a form accurate near u = 1
__device__ __forceinline__ float half_sweep(float u) { return atan2f(sqrtf(fmaxf(0.f, (1.f - u) * (1.f + u))), u); }

__device__ __forceinline__ void baseline(int kind, float al, float be, float a, float b, float &dth, float &dz,
                                         float &T) {
  dth = 0.f; dz = 0.f; T = 0.f;
  const float s = al < 0.0f ? -1.0f : 1.0f;
  const float kt = fabsf(cosf(be) * sinf(al)), kz = sinf(be);
  const float n = b / (b - a), kap = n * n;
  if (kind == 0) {
    const float kh = sqrtf(kap - kz * kz);
    const float u = kt / kh;  // p / b
    float sweep = half_sweep(u), lh = b * sqrtf(fmaxf(0.f, (1.f - u) * (1.f + u)));
    const float ua = u * (b / a);  // p / a
    if (ua <= 1.0f) {
      sweep -= half_sweep(ua);
      lh -= a * sqrtf(fmaxf(0.f, (1.f - ua) * (1.f + ua)));
    }
    dth = 2.0f * s * sweep;
    dz = 2.0f * lh * kz / kh;
    T = 2.0f * lh * kap / kh;
  } else if (kind == 3) {
    const float h = sqrtf(1.0f - kz * kz / kap);
    const float u = kt / h;
    dth = 2.0f * s * half_sweep(u);
    T = 2.0f * b * sqrtf(fmaxf(0.f, (1.f - u) * (1.f + u))) / h;
    dz = T * kz / kap;
  } else {
    const float p = b * kt, A = kap - kz * kz, kza2 = kz * kz * a * a;
    const float S = sqrtf(fmaf(A, p * p, kap * kza2));  // half the root of the discriminant of Q
    const float sq = b * cosf(al) * cosf(be);           // sqrt Q(b)
    const float sA = sqrtf(A);
    const float J0 = asinhf(sA * sq / S) / sA;          // int dx / sqrt Q from the root
    if (kind == 1) {                                    // x = u: Q = A u^2 - 2 a k_z^2 u - (p^2 + k_z^2 a^2)
      const float mC = fmaf(p, p, kza2), rm = sqrtf(mC);
      const float J1 = fmaf(a * kz * kz, J0, sq) / A;   // int u du / sqrt Q
      const float Jm = atan2f(rm * sq, fmaf(a * kz * kz, b - a, mC)) / rm;  // int du / (u sqrt Q)
      dth = 2.0f * s * p * Jm;
      dz = 2.0f * kz * (J1 + 2.0f * a * J0 + a * a * Jm);
      T = 2.0f * kap * J1;
    } else {                                            // x = r: Q = A r^2 - 2 kappa a r + kappa a^2 - p^2
      const float C = fmaf(kap * a, a, -p * p);
      const float y = C * sq * sq / (b * b * S * S);
      float g;                                          // asinh(sqrt y) / sqrt y
      if (fabsf(y) < 1e-3f) g = fmaf(y, fmaf(y, 0.075f, -1.0f / 6.0f), 1.0f);
      else if (y > 0.0f) g = asinhf(sqrtf(y)) / sqrtf(y);
      else g = asinf(sqrtf(-y)) / sqrtf(-y);
      const float Jm = sq / (b * S) * g;                // int dr / (r sqrt Q)
      const float J1 = fmaf(kap * a, J0, sq) / A;       // int r dr / sqrt Q
      dth = 2.0f * s * p * Jm;
      dz = 2.0f * kz * J1;
      T = 2.0f * kap * (J1 - 2.0f * a * J0 + a * a * Jm);
    }
  }
}

__device__ __forceinline__ int kind_of(float pol, float axis) {
  return (axis == 0.0f ? 0 : 2) + (pol == 0.0f ? 0 : 1);
}

__device__ __forceinline__ bool entry_ok(float phi, float z, float al, float be, float pol, float axis) {
  return isfinite(phi) && isfinite(z) && fabsf(al) < 0.5f * PI_F && fabsf(be) < 0.5f * PI_F &&
         (pol == 0.0f || pol == 1.0f) && (axis == 0.0f || axis == 1.0f);
}

// A model's job and the geometry it needs besides an entry: RT_SUR_SIDE
// (side-to-side transits of the infinite cylinder, no geometry) or
// RT_SUR_CAP (side entries whose path meets an end cap of the cloak with
// radii a < b and material height [z0, z1]).
struct JobP {
  int job;
  float a, b, z0, z1;
};

// Fraction u of the closed-form infinite-cylinder transit's rise that the
// entry's headroom allows: h / |dz_0| with h the distance from the entry
// height to the cap the ray climbs (or sinks) towards. z is monotonic along
// a transit (p_z keeps its sign), so the path meets that cap exactly when
// u < 1. Clamped to [0, 2] (u >= 1 never meets a cap).
__device__ __forceinline__ float cap_fraction(float z, float al, float be, int kind, const JobP &jp) {
  float dth0, dz0, T0;
  baseline(kind, al, be, jp.a, jp.b, dth0, dz0, T0);
  const float h = be >= 0.0f ? jp.z1 - z : z - jp.z0;
  const float u = h / fabsf(dz0);
  return u < 2.0f ? fmaxf(u, 0.0f) : 2.0f;  // NaN (dz_0 = 0 = h) -> 2
}

// Chord model of the path up to the cap, at rise fraction u, for the cap
// job's baselines. The infinite-cylinder path is symmetric about its
// turning point, which it reaches at u = 1/2, so it is modelled by the
// straight chord through the entry with the path's impact parameter w, the
// radius traversed at fraction u being sqrt(w^2 + (b^2 - w^2)(1 - 2u)^2):
//  - radial extraordinary and azimuthal ordinary branches: w the turning
//    radius, the larger root (kappa a + S) / (kappa - k_z^2) of the
//    quadratic Q of the closed-form transit (S as there);
//  - azimuthal extraordinary branch: the path is a straight line in
//    (rho = sqrt(kappa) (r - a), theta, zeta = sqrt(kappa) z) at unit speed
//    (Eq. (15)), so the chord in rho, with w = b k_theta / sqrt(1 - k_z^2 /
//    kappa) and rho_b = b, is exact, as are the sweep fraction and the
//    optical-path fraction u;
//  - radial ordinary branch: the straight chord (its paths never leave
//    through a cap: with n = 2 it is totally reflected at every cap).
// The swept azimuth is the chord's share frac of the whole sweep, the radial
// wave number at the modelled radius r_c comes from the dispersion relation
// k_r^2 / m_r + k_theta^2 / m_theta + k_z^2 / m_z = 1 (k_theta = p_theta /
// r_c, k_z conserved; the metric of Eqs. (14)/(15): m = kappa (1, 1, 1),
// kappa (1, s, s), kappa s (1, 1, 1), kappa (1, s, 1) for the radial o, e
// and azimuthal o, e branches, s = ((r - a) / r)^2) with the sign of the leg
// (inwards before the turning point), and it is the vacuum direction's d_r
// after the cap (tangential continuity, Sect. 3), with |d_z| from
// normalization.
__device__ __forceinline__ void cap_chord(int kind, float al, float be, float u, float a, float b, float &frac,
                                          float &rc, float &dr, float &adz) {
  const float kap = (b / (b - a)) * (b / (b - a)), skap = b / (b - a);
  const float kt = fabsf(cosf(be) * sinf(al)), kz = sinf(be), p = b * kt;
  const float A = kap - kz * kz;
  float w;
  if (kind == 3) {
    w = b * kt / sqrtf(1.0f - kz * kz / kap);
  } else if (kind == 0) {
    w = p / sqrtf(A);
  } else {
    w = (kap * a + sqrtf(fmaf(A, p * p, kap * kz * kz * a * a))) / A;
  }
  w = fminf(w, b);
  const float v = 1.0f - 2.0f * u;
  const float wb = sqrtf(fmaxf(0.0f, (b - w) * (b + w)));
  const float rr = sqrtf(fmaf(wb * wb, v * v, w * w));
  rc = kind == 3 ? a + rr / skap : rr;
  const float half = atan2f(wb, w);
  frac = half > 1e-6f ? 0.5f * (1.0f - atan2f(wb * v, w) / half) : u;
  // k_r^2 vanishes at the turning point, where its terms cancel; written
  // with the factor rr - w = wb^2 v^2 / (rr + w) taken out it is v^2 times a
  // smooth positive function, so d_r = -v (...) runs linearly through it:
  //  - radial ordinary, azimuthal extraordinary (straight in r or rho):
  //    k_r^2 = (kappa - k_z^2)(rr^2 - w^2) / rr^2;
  //  - radial extraordinary, azimuthal ordinary: k_r^2 = m_r Q(r) /
  //    (kappa (r - a)^2) with Q = (kappa - k_z^2)(r - w)(r - r_s), r_s the
  //    smaller root (kappa a^2 - p^2) / ((kappa - k_z^2) w).
  if (kind == 0 || kind == 3) {
    dr = -v * wb * sqrtf(A) / rr;
  } else {
    const float rs = (kap * a * a - p * p) / (A * w);
    const float g = sqrtf(fmaxf(0.0f, A * (rc - rs) / (rc + w)));
    dr = -v * wb * g / (kind == 1 ? rc - a : rc);
  }
  const float kth = p / rc;
  adz = sqrtf(fmaxf(0.0f, 1.0f - dr * dr - kth * kth));
}

// Network input features of entry i. The transit of the infinite cylinder
// is invariant under rotation about and translation along its axis, so the
// exit offsets do not depend on phi or z; those two slots carry instead the
// entry's tangential wave numbers k_theta = cos(beta) sin(alpha) and
// k_z = sin(beta), the invariants p_theta / r2 and p_z of the transit:
//   side job: f = (k_theta, k_z, alpha, beta, branch bit, axis bit).
// A path that meets a cap depends on the height as well; the cloak is also
// symmetric under the mirror z -> z0 + z1 - z, which flips beta, so the cap
// job takes |k_z| and the cap fraction u (cap_fraction) instead:
//   cap job:  f = (k_theta, |k_z|, u, alpha, branch bit, axis bit).
__device__ __forceinline__ void features(const float *__restrict__ x6, long long ld, long long i, const JobP &jp,
                                         float f[NIN]) {
  const float al = x6[2 * ld + i], be = x6[3 * ld + i];
  f[0] = cosf(be) * sinf(al);
  f[1] = sinf(be);
  f[2] = al;
  f[3] = be;
  f[4] = x6[4 * ld + i];
  f[5] = x6[5 * ld + i];
  if (jp.job == RT_SUR_CAP) {
    f[1] = fabsf(f[1]);
    f[2] = cap_fraction(x6[ld + i], al, be, kind_of(f[4], f[5]), jp);
    f[3] = al;
  }
}

// standardized outputs (n x 5) -> SoA targets (5 x ld)
__global__ void k_destd(const float *__restrict__ y, int n, long long ld, const float *__restrict__ sc,
                        float *__restrict__ t) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * NOUT) return;
  const int row = (int)(i / NOUT), o = (int)(i - (long long)row * NOUT);
  t[o * ld + row] = fmaf(y[i], sc[S_OSTD + o], sc[S_OMEAN + o]);
}

// backward of layer 5 (FP32): dW5 = a4^T dy, db5 = sum dy, with a4 =
// silu(z4) recomputed from the saved pre-activation (the same FP32 function
// as the forward's), dz4 = (dy W5^T) * silu'(z4) -> BF16 for the next
// product (row-major and transposed), and db4 = sum dz4 (FP32). A block
// takes a run of rows in chunks of 64, wave w rows 16 w .. 16 w + 15 of a
// chunk, lane l units 4 l .. 4 l + 3 (one 16-byte load per lane covers a
// row's 256 units); the transposed copy goes through LDS and out in whole
// 128-byte lines. Each block writes its partial sums of the 1,541 gradient
// entries b4 [256], W5 [256][5], b5 [5] (contiguous in the parameter vector
// from OFF_B4) to a row of `part`.
constexpr int L5_N = HID + HID * NOUT + NOUT, L5_LD = 1544, L5_MAXB = 1024;
static_assert(OFF_W5 == OFF_B4 + HID && OFF_B5 == OFF_W5 + HID * NOUT, "b4, W5, b5 are contiguous");

__global__ void __launch_bounds__(256) k_layer5_back(const float *__restrict__ dy, const float *__restrict__ z4,
                                                     int n, const float *__restrict__ P, float *__restrict__ part,
                                                     bf16 *__restrict__ dzb, bf16 *__restrict__ dzT, long long ldT) {
  // unit u's 8 pieces of 8 rows of a chunk at tp[9 u + p]; afterwards the
  // same memory holds the 4 waves' partial sums
  __shared__ bf16x8 tp[HID * 9];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int u0 = 4 * lane;
  float w5[4][NOUT], gw[4][NOUT], gz[4] = {0.f, 0.f, 0.f, 0.f}, gb[NOUT];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      w5[i][o] = P[OFF_W5 + (u0 + i) * NOUT + o];
      gw[i][o] = 0.0f;
    }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) gb[o] = 0.0f;
  const int per = (((n + gridDim.x - 1) / gridDim.x) + 63) & ~63;
  const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
  for (int c0 = r0; c0 < r1; c0 += 64) {
    const int c1 = min(r1, c0 + 64);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int rb = c0 + 16 * w + 8 * p;
      // the 8 rows' loads together (rows past the chunk repeat its last
      // row and are not used)
      float4 zz[8];
      float d[8][NOUT];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const long long row = min(rb + k, c1 - 1);
        zz[k] = *reinterpret_cast<const float4 *>(&z4[row * HID + u0]);
#pragma unroll
        for (int o = 0; o < NOUT; ++o) d[k][o] = dy[row * NOUT + o];
      }
      bf16x8 pk[4];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float zk[4] = {zz[k].x, zz[k].y, zz[k].z, zz[k].w};
        bf16x4 out;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float a = silu_f(zk[i]);
          float da = 0.f;
#pragma unroll
          for (int o = 0; o < NOUT; ++o) da = fmaf(d[k][o], w5[i][o], da);
          const float g = da * dsilu_f(zk[i]);
          out[i] = (bf16)g;
          pk[i][k] = out[i];
          if (rb + k < c1) {
            gz[i] += g;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) gw[i][o] = fmaf(a, d[k][o], gw[i][o]);
          }
        }
        if (rb + k < c1) {
#pragma unroll
          for (int o = 0; o < NOUT; ++o) gb[o] += d[k][o];
          *reinterpret_cast<bf16x4 *>(&dzb[(long long)(rb + k) * HID + u0]) = out;
        }
      }
      if (rb < c1) {
#pragma unroll
        for (int i = 0; i < 4; ++i) tp[9 * (u0 + i) + ((rb - c0) >> 3)] = pk[i];
      }
    }
    __syncthreads();
    for (int e = tid; e < 8 * HID; e += 256) {
      const int u = e >> 3, p = e & 7, row = c0 + 8 * p;
      if (row >= c1) continue;
      const bf16x8 v = tp[9 * u + p];
      bf16 *o = dzT + (long long)u * ldT + row;
      if (row + 8 <= c1) {
        *reinterpret_cast<bf16x8 *>(o) = v;
      } else {
        for (int k = 0; row + k < c1; ++k) o[k] = v[k];
      }
    }
    __syncthreads();
  }
  // the 4 waves' sums: [wave][unit][W5 row (5), b4], then db5 [wave][5]
  float *red = reinterpret_cast<float *>(tp);
  static_assert((4 * HID * (NOUT + 1) + 4 * NOUT) * sizeof(float) <= sizeof(tp), "reduction fits");
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int o = 0; o < NOUT; ++o) red[(w * HID + u0 + i) * (NOUT + 1) + o] = gw[i][o];
    red[(w * HID + u0 + i) * (NOUT + 1) + NOUT] = gz[i];
  }
  if (lane == 0) {
#pragma unroll
    for (int o = 0; o < NOUT; ++o) red[4 * HID * (NOUT + 1) + w * NOUT + o] = gb[o];
  }
  __syncthreads();
  float *pb = part + (long long)blockIdx.x * L5_LD;
  for (int e = tid; e < HID * (NOUT + 1); e += 256) {
    const int u = e / (NOUT + 1), k = e % (NOUT + 1);
    constexpr int WS = HID * (NOUT + 1);
    const float v = (red[e] + red[WS + e]) + (red[2 * WS + e] + red[3 * WS + e]);
    pb[k == NOUT ? u : HID + u * NOUT + k] = v;
  }
  if (tid < NOUT) {
    const float *rb = red + 4 * HID * (NOUT + 1);
    pb[HID + HID * NOUT + tid] = (rb[tid] + rb[NOUT + tid]) + (rb[2 * NOUT + tid] + rb[3 * NOUT + tid]);
  }
}

__global__ void k_fill(float *p, long long n, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u32(unsigned int *p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__device__ __forceinline__ bool is_bias(long long i) {
  return (i >= OFF_B1 && i < OFF_W2) || (i >= OFF_B2 && i < OFF_W3) || (i >= OFF_B3 && i < OFF_W4) ||
         (i >= OFF_B4 && i < OFF_W5) || i >= OFF_B5;
}

// index of FP32 parameter i in the transposed BF16 copy (-1: no copy);
// its row-major copy sits at NBF + (layer offset + e)
__device__ __forceinline__ long long bf16_index(long long i, long long &rowmajor) {
  long long l, e;
  if (i >= OFF_W2 && i < OFF_B2) { l = 0; e = i - OFF_W2; }
  else if (i >= OFF_W3 && i < OFF_B3) { l = 1; e = i - OFF_W3; }
  else if (i >= OFF_W4 && i < OFF_B4) { l = 2; e = i - OFF_W4; }
  else return -1;
  const long long in = e / HID, out = e - in * HID;
  rowmajor = NBF + l * HID * HID + e;
  return l * HID * HID + out * HID + in;
}

// AdamW (decoupled weight decay on the weights, not the biases) on the FP32
// master weights, then the BF16 copy of each updated W2..W4 entry
__global__ void k_adamw(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ m,
                        float *__restrict__ v, bf16 *__restrict__ Pb, float lr, float wd, float b1, float b2,
                        float c1, float c2, float eps) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const float g = G[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  float p = P[i];
  if (!is_bias(i)) p -= lr * wd * p;
  p -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  P[i] = p;
  long long kr;
  const long long k = bf16_index(i, kr);
  if (k >= 0) {
    Pb[k] = (bf16)p;
    Pb[kr] = (bf16)p;
  }
}

__global__ void k_refresh_bf16(const float *__restrict__ P, bf16 *__restrict__ Pb) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  long long kr;
  const long long k = bf16_index(i, kr);
  if (k >= 0) {
    Pb[k] = (bf16)P[i];
    Pb[kr] = (bf16)P[i];
  }
}

// masked first and second moments of the 6 input features and 5 targets (FP64 sums)
constexpr int NMOM = 2 * (NIN + NOUT) + 1;
__global__ void __launch_bounds__(256) k_moments(const float *__restrict__ x, const float *__restrict__ t, long long ld,
                                                 const float *__restrict__ wrow, int n, JobP jp,
                                                 double *__restrict__ acc) {
  double s[NMOM];
#pragma unroll
  for (int k = 0; k < NMOM; ++k) s[k] = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double wr = wrow ? wrow[i] : 1.0;
    if (wr == 0.0) continue;
    s[NMOM - 1] += wr;
    float f[NIN];
    features(x, ld, i, jp, f);
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      const double v = f[k];
      s[2 * k] += wr * v;
      s[2 * k + 1] += wr * v * v;
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      const double v = t[o * ld + i];
      s[2 * (NIN + o)] += wr * v;
      s[2 * (NIN + o) + 1] += wr * v * v;
    }
  }
#pragma unroll
  for (int k = 0; k < NMOM; ++k) {
    double v = s[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(&acc[k], v);
  }
}

__global__ void k_fill_f64(double *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// exit point and unit direction from exit parameters
__device__ __forceinline__ void exit_ray(const float *p, float b, float x[3], float d[3]) {
  float sp, cp, sa, ca, sb, cbt;
  sincosf(p[0], &sp, &cp);
  sincosf(p[2], &sa, &ca);
  sincosf(p[3], &sb, &cbt);
  x[0] = b * cp; x[1] = b * sp; x[2] = p[1];
  d[0] = cbt * (ca * cp - sa * sp);
  d[1] = cbt * (ca * sp + sa * cp);
  d[2] = sb;
}

__global__ void __launch_bounds__(256) k_encode(const float *__restrict__ x6, const float *__restrict__ y5,
                                                const int *__restrict__ status, long long ld, long long n, float a,
                                                float b, float *__restrict__ t5, float *__restrict__ wrow) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float phi = x6[i], z = x6[ld + i], al = x6[2 * ld + i], be = x6[3 * ld + i];
  const float pol = x6[4 * ld + i], axis = x6[5 * ld + i];
  float t[NOUT] = {0.f, 0.f, 0.f, 0.f, 0.f};
  bool ok = status[i] == RT_RAY_EXITED && entry_ok(phi, z, al, be, pol, axis);
  if (ok) {
    const float s = al < 0.0f ? -1.0f : 1.0f;
    const float dth = s * wrap2pi(s * (y5[i] - phi));
    float dth0, dz0, T0;
    baseline(kind_of(pol, axis), al, be, a, b, dth0, dz0, T0);
    t[0] = dth - dth0;
    t[1] = (y5[ld + i] - z) - dz0;
    t[2] = y5[2 * ld + i] - al;
    t[3] = y5[3 * ld + i] - be;
    t[4] = y5[4 * ld + i] - T0;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) ok = ok && isfinite(t[o]);
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) t5[o * ld + i] = ok ? t[o] : 0.0f;
  wrow[i] = ok ? 1.0f : 0.0f;
}

// Cap-job targets. A side entry whose path leaves through an end cap exits
// as the vacuum ray from its cap point, given where that ray crosses r = b;
// the straight vacuum leg back to the cap plane recovers the cap point
// (r_c, theta_c) and the optical path T_c up to it. The cap's refraction
// keeps the tangential wave vector (k_r, k_theta), so the vacuum direction
// there has d_theta = b k_theta / r_c (the conserved angular momentum) and
// |d_z| from normalization: the exit is fixed by (theta_c, r_c, d_r, T_c).
// With u the cap fraction (cap_fraction) and (dtheta_0, T_0) the closed-form
// transit of the infinite cylinder, whose share u the path covers before the
// cap in rise, the state (dtheta_c, r_c, d_r, T_c) and |d_z| (a second
// estimate, checked against the normalization by the gate) enter as
// residuals,
// dtheta_c the signed azimuth swept from the entry to the cap point (sign of
// alpha), each against the chord model of the path (cap_chord):
//   t0 = dtheta_c - frac dtheta_0,  t1 = r_c - r_c^chord,
//   t2 = d_r - d_r^chord,           t3 = T_c - u T_0,
//   t4 = |d_z| - |d_z|^chord.
// Rows that do not leave through the cap they head for get w = 0.
__global__ void __launch_bounds__(256) k_encode_cap(const float *__restrict__ x6, const float *__restrict__ y5,
                                                    const int *__restrict__ status, long long ld, long long n,
                                                    JobP jp, float *__restrict__ t5, float *__restrict__ wrow) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float phi = x6[i], z = x6[ld + i], al = x6[2 * ld + i], be = x6[3 * ld + i];
  const float pol = x6[4 * ld + i], axis = x6[5 * ld + i];
  float t[NOUT] = {0.f, 0.f, 0.f, 0.f, 0.f};
  const float ze = y5[ld + i];
  const bool up = be >= 0.0f;
  bool ok = status[i] == RT_RAY_EXITED && entry_ok(phi, z, al, be, pol, axis) && z >= jp.z0 && z <= jp.z1 &&
            (up ? ze > jp.z1 : ze < jp.z0);
  if (ok) {
    float ex[NOUT], xe[3], de[3];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) ex[o] = y5[o * ld + i];
    exit_ray(ex, jp.b, xe, de);
    const float tb = (xe[2] - (up ? jp.z1 : jp.z0)) / de[2];  // vacuum leg back to the cap plane
    const float cx = fmaf(-tb, de[0], xe[0]), cy = fmaf(-tb, de[1], xe[1]);
    const float rc = sqrtf(fmaf(cx, cx, cy * cy));
    const float s = al < 0.0f ? -1.0f : 1.0f;
    float dth = s * wrap2pi(s * (atan2f(cy, cx) - phi));
    if (s * dth > 2.0f * PI_F - 1e-3f) dth -= s * 2.0f * PI_F;  // a sweep rounded to just below zero
    const int kind = kind_of(pol, axis);
    float dth0, dz0, T0;
    baseline(kind, al, be, jp.a, jp.b, dth0, dz0, T0);
    const float u = cap_fraction(z, al, be, kind, jp);
    float frac, rcb, drb, adzb;
    cap_chord(kind, al, be, u, jp.a, jp.b, frac, rcb, drb, adzb);
    t[0] = fmaf(-frac, dth0, dth);
    t[1] = rc - rcb;
    t[2] = fmaf(cx, de[0], cy * de[1]) / rc - drb;
    t[3] = fmaf(-u, T0, ex[4] - tb);
    t[4] = fabsf(de[2]) - adzb;
    ok = tb >= 0.0f && u < 1.0f;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) ok = ok && isfinite(t[o]);
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) t5[o * ld + i] = ok ? t[o] : 0.0f;
  wrow[i] = ok ? 1.0f : 0.0f;
}

// standardized network outputs -> exit parameters (phi', z', alpha', beta', T)
__device__ __forceinline__ void decode(const float *yrow, const float *sc, float phi, float z, float al, float be,
                                       int kind, float a, float b, float out[NOUT]) {
  float t[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) t[o] = fmaf(yrow[o], sc[S_OSTD + o], sc[S_OMEAN + o]);
  float dth0, dz0, T0;
  baseline(kind, al, be, a, b, dth0, dz0, T0);
  out[0] = wrap2pi(phi + t[0] + dth0);
  out[1] = z + (dz0 + t[1]);
  out[2] = al + t[2];
  out[3] = be + t[3];
  out[4] = T0 + t[4];
}

// Cap-job prediction -> exit parameters: the cap point and the vacuum
// direction from the targets of k_encode_cap, then the straight vacuum leg
// to r = b. Returns false where the prediction is no usable cap exit: a cap
// point within `margin` of the rims r = a, r = b of the cap, a vacuum
// direction within |d_z| < 0.05 of grazing the cap (the refraction is
// ill-conditioned next to total reflection) or with a horizontal speed
// below 0.05 (a vacuum leg longer than ~2 b / 0.05), or the two estimates
// of |d_z| (normalization, output t4) apart by more than CAP_DZ_CHECK: a
// network that contradicts itself that much is outside what it learned.
constexpr float CAP_DZ_CHECK = 1e-2f;
__device__ __forceinline__ bool decode_cap(const float *yrow, const float *sc, float phi, float z, float al,
                                           float be, int kind, const JobP &jp, float margin, float out[NOUT]) {
  float t[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) t[o] = fmaf(yrow[o], sc[S_OSTD + o], sc[S_OMEAN + o]);
  float dth0, dz0, T0;
  baseline(kind, al, be, jp.a, jp.b, dth0, dz0, T0);
  const float u = cap_fraction(z, al, be, kind, jp);
  float frac, rcb, drb, adzb;
  cap_chord(kind, al, be, u, jp.a, jp.b, frac, rcb, drb, adzb);
  const bool up = be >= 0.0f;
  const float thc = phi + fmaf(frac, dth0, t[0]);
  const float rc = rcb + t[1], dr = drb + t[2];
  const float dt = jp.b * cosf(be) * sinf(al) / rc;
  const float q = fmaf(dr, dr, dt * dt);  // horizontal speed squared
  const float adz = sqrtf(fmaxf(0.0f, 1.0f - q));
  float st, ct;
  sincosf(thc, &st, &ct);
  const float cx = rc * ct, cy = rc * st;
  const float dx = dr * ct - dt * st, dy = dr * st + dt * ct;
  // vacuum leg: |(c + s d)_xy| = b with s > 0 from a cap point inside
  // (r_c < b), in the form without cancellation for either sign of d_r
  const float qb = rc * dr, qc = (rc - jp.b) * (rc + jp.b);
  const float disc = sqrtf(fmaxf(0.0f, fmaf(qb, qb, -q * qc)));
  const float s = qb >= 0.0f ? -qc / (qb + disc) : (disc - qb) / q;
  const float px = fmaf(s, dx, cx), py = fmaf(s, dy, cy);
  const float ph = wrap2pi(atan2f(py, px));
  float sph, cph;
  sincosf(ph, &sph, &cph);
  out[0] = ph;
  out[1] = fmaf(s, up ? adz : -adz, up ? jp.z1 : jp.z0);
  out[2] = atan2f(dy * cph - dx * sph, fmaf(dx, cph, dy * sph));
  out[3] = up ? asinf(fminf(1.0f, adz)) : -asinf(fminf(1.0f, adz));
  out[4] = fmaf(u, T0, t[3]) + s;
  return rc > jp.a + margin && rc < jp.b - margin && adz >= 0.05f && q >= 0.0025f &&
         fabsf(adzb + t[4] - adz) <= CAP_DZ_CHECK;
}

// cell of the side job's trust map: (axis, branch) x alpha x beta
__device__ __forceinline__ int cell_of(int kind, float al, float be) {
  int ia = (int)floorf((al + 0.5f * PI_F) * (NCELL_A / PI_F));
  int ib = (int)floorf((be + 0.5f * PI_F) * (NCELL_B / PI_F));
  ia = min(max(ia, 0), NCELL_A - 1);
  ib = min(max(ib, 0), NCELL_B - 1);
  return (kind * NCELL_A + ia) * NCELL_B + ib;
}

// cell of the cap job's trust map: (axis, branch) x alpha x |beta| x u
__device__ __forceinline__ int cell_cap(int kind, float al, float be, float u) {
  int ia = (int)floorf((al + 0.5f * PI_F) * (CAP_A / PI_F));
  int ib = (int)floorf(fabsf(be) * (2.0f * CAP_B / PI_F));
  int iu = (int)floorf(u * (float)CAP_U);
  ia = min(max(ia, 0), CAP_A - 1);
  ib = min(max(ib, 0), CAP_B - 1);
  iu = min(max(iu, 0), CAP_U - 1);
  return ((kind * CAP_A + ia) * CAP_B + ib) * CAP_U + iu;
}

struct GateP {
  float a, b, z0, z1;  // cloak radii r1, r2 and material height range
  float hres_max;    // conservation residual limit
  float cap_margin;  // distance of the predicted exit height from a cap (side job), of the cap point from the rims (cap job)
  float p_min;       // near-singular band of the conserved wave number
};

// Outside the near-singular band: the conserved wave number that keeps the
// path away from r = a (k_theta for the azimuthal cloak's extraordinary
// branch, whose metric is singular in theta only; |(k_theta, k_z)| for the
// radial extraordinary and azimuthal ordinary branches, singular in theta
// and z; the radial cloak's ordinary branch is homogeneous) is >= p_min.
__device__ __forceinline__ bool outside_band(int kind, float al, float be, float p_min) {
  if (kind == 0 || !(p_min > 0.0f)) return true;
  const float kt = cosf(be) * sinf(al), kz = sinf(be);
  const float p = kind == 3 ? fabsf(kt) : sqrtf(fmaf(kt, kt, kz * kz));
  return p >= p_min;
}

// The input half of the gate: a valid entry inside the material's height
// range, outside the near-singular band, in a trusted cell of the model's
// trust map and, for the cap job, heading for a cap (u < 1).
__device__ __forceinline__ bool gate_inputs(float phi, float z, float al, float be, float pol, float axis,
                                            const unsigned char *__restrict__ map, const GateP &gp, const JobP &jp) {
  if (!(entry_ok(phi, z, al, be, pol, axis) && z >= gp.z0 && z <= gp.z1)) return false;
  const int kind = kind_of(pol, axis);
  if (!outside_band(kind, al, be, gp.p_min)) return false;
  if (jp.job == RT_SUR_CAP) {
    const float u = cap_fraction(z, al, be, kind, jp);
    return u < 1.0f && map[cell_cap(kind, al, be, u)] != 0;
  }
  return map[cell_of(kind, al, be)] != 0;
}

// Gate and write the accepted predictions. A prediction is rejected (and
// the exact integrator traces the ray) when its input fails gate_inputs or
//  - side job: the predicted exit ray violates the conservation of the
//    tangential wave numbers (p_theta / b and p_z, equal at entry and exit
//    on r = b for every side-to-side transit) by more than hres_max, or the
//    predicted exit height lies within cap_margin of an end cap or beyond
//    it (z is monotonic along a transit since p_z keeps its sign, so an exit
//    height inside the material with margin means the whole path stayed
//    inside);
//  - cap job: the prediction is no usable cap exit (decode_cap).
__device__ __forceinline__ void gate_row(long long i, const float *__restrict__ x6, long long ld,
                                         const float *yrow, const float *__restrict__ sc,
                                         const unsigned char *__restrict__ map, const GateP &gp, const JobP &jp,
                                         float *__restrict__ y5, unsigned char *__restrict__ fallback,
                                         int *__restrict__ status) {
  const float phi = x6[i], z = x6[ld + i], al = x6[2 * ld + i], be = x6[3 * ld + i];
  const float pol = x6[4 * ld + i], axis = x6[5 * ld + i];
  bool acc = gate_inputs(phi, z, al, be, pol, axis, map, gp, jp);
  float out[NOUT];
  if (acc) {
    const int kind = kind_of(pol, axis);
    if (jp.job == RT_SUR_CAP) {
      acc = decode_cap(yrow, sc, phi, z, al, be, kind, jp, gp.cap_margin, out);
    } else {
      decode(yrow, sc, phi, z, al, be, kind, gp.a, gp.b, out);
      const float kt = cosf(be) * sinf(al), kz = sinf(be);
      const float kt2 = cosf(out[3]) * sinf(out[2]), kz2 = sinf(out[3]);
      const float res = fmaxf(fabsf(kt2 - kt), fabsf(kz2 - kz));
      acc = res <= gp.hres_max && out[1] >= gp.z0 + gp.cap_margin && out[1] <= gp.z1 - gp.cap_margin;
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) acc = acc && isfinite(out[o]);
  }
  fallback[i] = acc ? 0 : 1;
  if (acc) {
#pragma unroll
    for (int o = 0; o < NOUT; ++o) y5[o * ld + i] = out[o];
    status[i] = RT_RAY_EXITED;
  }
}

// First half of the gate, on the inputs alone: entries that pass
// gate_inputs are appended to idx for the network; the others go to the
// exact transit (fallback = 1). With `chained`, only the rows an earlier
// model rejected (fallback != 0) are considered; the others keep fallback 0.
__global__ void __launch_bounds__(256) k_pregate(const float *__restrict__ x6, long long ld, int n,
                                                 const unsigned char *__restrict__ map, GateP gp, JobP jp,
                                                 int chained, unsigned char *__restrict__ fallback,
                                                 int *__restrict__ idx, unsigned int *__restrict__ count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool take = false;
  if (i < n && (!chained || fallback[i] != 0)) {
    take = gate_inputs(x6[i], x6[ld + i], x6[2 * ld + i], x6[3 * ld + i], x6[4 * ld + i], x6[5 * ld + i], map, gp,
                       jp);
    fallback[i] = take ? 0 : 1;
  }
  const unsigned long long m = __ballot(take);
  unsigned int base = 0;
  if (m != 0ull) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    if ((int)__lane_id() == leader) base = atomicAdd(count, (unsigned int)__popcll(m));
    base = __shfl(base, leader);
  }
  const unsigned int lane = __lane_id();
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  if (take) idx[base + (unsigned int)__popcll(m & below)] = (int)i;
}

// second half of the gate on the network's outputs of the compacted entries
__global__ void __launch_bounds__(256) k_gate_idx(const float *__restrict__ x6, long long ld,
                                                  const int *__restrict__ idx, const unsigned int *count,
                                                  const float *__restrict__ y, const float *__restrict__ sc,
                                                  const unsigned char *__restrict__ map, GateP gp, JobP jp,
                                                  float *__restrict__ y5, unsigned char *__restrict__ fallback,
                                                  int *__restrict__ status) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < (long long)*count) gate_row(idx[p], x6, ld, y + p * NOUT, sc, map, gp, jp, y5, fallback, status);
}

// ---------------------------------------------------------------------------
// Fused inference: the whole network for FR rows per block, activations
// resident in LDS (BF16, FR x 256, rows padded to 264 so that the 16 rows
// an operand read touches fall in distinct banks). Each hidden layer is
// computed transposed, out^T = W^T act^T, so that an MFMA 16x16x32 tile's
// A operand is 8 consecutive inputs of one output unit (one 16-byte load of
// the transposed BF16 weights, streamed from L2), its B operand 8
// consecutive inputs of one row (one 16-byte LDS read), and each lane's 4
// results are 4 consecutive output units of one row (one 8-byte LDS store).
// Wave w owns output units 64w..64w+63: 4 unit tiles x 8 row tiles, 128 FP32
// accumulators per lane. Layer 1 (FP32) fills the tile; layer 5 (FP32)
// reduces the layer-4 accumulators over each lane's 16 units, across the 4
// lane groups of a wave, then across the 4 waves through LDS, and the block
// writes the standardized outputs (n x 5).
// ---------------------------------------------------------------------------
constexpr int FR = 128, ALD = HID + 8;

// copy the block's BF16 activation tile (R rows of ALD, padded)
// transposed to dst[unit * ldT + row0 + r]: 8 consecutive rows of one unit
// per 16-byte store, R / 8 consecutive threads on the consecutive pieces of
// one unit (whole 128-byte lines per group of 8 lanes at R = 64)
template <int R>
__device__ __forceinline__ void store_act_tile_t(const bf16 *act, bf16 *__restrict__ dst, long long ldT,
                                                 long long row0, int n, int tid) {
  constexpr int P8 = R / 8;
#pragma unroll 2
  for (int e = tid; e < P8 * HID; e += 256) {
    const int u = e / P8, r8 = (e % P8) * 8;
    bf16 *o = dst + (long long)u * ldT + row0 + r8;
    if (row0 + r8 + 8 <= n) {
      bf16x8 pk;
#pragma unroll
      for (int k = 0; k < 8; ++k) pk[k] = act[(r8 + k) * ALD + u];
      *reinterpret_cast<bf16x8 *>(o) = pk;
    } else {
      for (int k = 0; row0 + r8 + k < n; ++k) o[k] = act[(r8 + k) * ALD + u];
    }
  }
}

// What the training forward keeps for the backward pass, per row of the
// batch (row-major [n][256] unless noted): the standardized features xf
// [n][6], the pre-activations z1..z4 (FP32), the BF16 activations a1..a3
// (the inputs of the BF16 layers) transposed, aT[l][unit * ldT + row] (the
// weight-gradient products read them along the batch), and, instead of the
// standardized outputs,
// the loss term and its gradient dy [n][5] against the targets t (SoA 5 x
// ld) with the row weights w (NULL = 1): per element d = y - (t - out_mean)
// / out_std, the loss d^2, or for huber = delta > 0 the Huber function (d^2
// up to |d| = delta, then 2 delta |d| - delta^2, gradient clipped to
// 2 delta sign(d)), times the row weight; loss and gradient divided by n.
struct TrainSink {
  float *xf;
  float *z[4];
  bf16 *aT[3];
  long long ldT;
  const float *t;
  long long ldt;
  const float *w;
  float huber;
  float *dy;
  float *loss;
};

// With idx != NULL, row r of the network is entry idx[r] for r < *count
// (a compacted subset); otherwise row r is entry r, r < n.
__global__ void __launch_bounds__(256, 2) k_mlp_fused(const float *__restrict__ x6, long long ld, int n,
                                                      const int *__restrict__ idx, const unsigned int *count,
                                                      const float *__restrict__ P, const bf16 *__restrict__ Wt,
                                                      const float *__restrict__ sc, JobP jp,
                                                      float *__restrict__ yout) {
  __shared__ __attribute__((aligned(16))) bf16 act[FR * ALD];
  __shared__ float xn[FR * NIN];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const long long row0 = (long long)blockIdx.x * FR;
  if (idx) n = (int)*count;  // block-uniform
  if (row0 >= n) return;
  // standardized input features of the tile (rows past n read as zeros)
  if (tid < FR) {
    const long long i = row0 + tid;
    float f[NIN] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < n) {
      features(x6, ld, idx ? (long long)idx[i] : i, jp, f);
#pragma unroll
      for (int k = 0; k < NIN; ++k) f[k] = (f[k] - sc[S_INOFF + k]) * sc[S_INSCALE + k];
    }
#pragma unroll
    for (int k = 0; k < NIN; ++k) xn[tid * NIN + k] = f[k];
  }
  __syncthreads();
  {  // layer 1 (FP32): thread = pair of hidden units x half of the rows
    const int u = 2 * (tid & 127), rb = (tid >> 7) * (FR / 2);
    float w0[NIN], w1[NIN];
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      w0[k] = P[OFF_W1 + k * HID + u];
      w1[k] = P[OFF_W1 + k * HID + u + 1];
    }
    const float b0 = P[OFF_B1 + u], b1 = P[OFF_B1 + u + 1];
    for (int r = rb; r < rb + FR / 2; ++r) {
      float z0 = b0, z1 = b1;
#pragma unroll
      for (int k = 0; k < NIN; ++k) {
        z0 = fmaf(xn[r * NIN + k], w0[k], z0);
        z1 = fmaf(xn[r * NIN + k], w1[k], z1);
      }
      bf16x2 pr;
      pr[0] = (bf16)silu_f(z0);
      pr[1] = (bf16)silu_f(z1);
      *reinterpret_cast<bf16x2 *>(&act[r * ALD + u]) = pr;
    }
  }
  __syncthreads();
  const int q = lane >> 4, c16 = lane & 15, ub = 64 * w;
  const long long offb[3] = {OFF_B2, OFF_B3, OFF_B4};
  f32x4 acc[4][8];  // [unit tile][row tile]
  for (int l = 0; l < 3; ++l) {
    const bf16 *W = Wt + (long long)l * HID * HID;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 8; ++tj) acc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int k0 = 0; k0 < HID; k0 += 32) {
      bf16x8 aop[4];
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
        aop[ti] = *reinterpret_cast<const bf16x8 *>(W + (ub + 16 * ti + c16) * HID + k0 + 8 * q);
#pragma unroll
      for (int tj = 0; tj < 8; ++tj) {
        const bf16x8 bop = *reinterpret_cast<const bf16x8 *>(&act[(16 * tj + c16) * ALD + k0 + 8 * q]);
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[ti], bop, acc[ti][tj], 0, 0, 0);
      }
    }
    __syncthreads();  // every wave has read the layer's input tile
    if (l < 2) {
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) {
        const int u0 = ub + 16 * ti + 4 * q;  // this lane's 4 consecutive units
        float bias[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) bias[r] = P[offb[l] + u0 + r];
#pragma unroll
        for (int tj = 0; tj < 8; ++tj) {
          bf16x4 pk;
#pragma unroll
          for (int r = 0; r < 4; ++r) pk[r] = (bf16)silu_f(acc[ti][tj][r] + bias[r]);
          *reinterpret_cast<bf16x4 *>(&act[(16 * tj + c16) * ALD + u0]) = pk;
        }
      }
      __syncthreads();
    } else {
      // layer 5 (FP32) on a4 = silu(z4): partial sums over this lane's 16
      // units for each of its 8 rows, then over the 4 lane groups
      float s5[8][NOUT];
#pragma unroll
      for (int tj = 0; tj < 8; ++tj)
#pragma unroll
        for (int o = 0; o < NOUT; ++o) s5[tj][o] = 0.0f;
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) {
        const int u0 = ub + 16 * ti + 4 * q;
        float bias[4], w5[4][NOUT];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          bias[r] = P[offb[l] + u0 + r];
#pragma unroll
          for (int o = 0; o < NOUT; ++o) w5[r][o] = P[OFF_W5 + (u0 + r) * NOUT + o];
        }
#pragma unroll
        for (int tj = 0; tj < 8; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float a4 = silu_f(acc[ti][tj][r] + bias[r]);
#pragma unroll
            for (int o = 0; o < NOUT; ++o) s5[tj][o] = fmaf(a4, w5[r][o], s5[tj][o]);
          }
      }
      float *red = reinterpret_cast<float *>(act);  // [4 waves][FR][NOUT]
#pragma unroll
      for (int tj = 0; tj < 8; ++tj) {
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
          s5[tj][o] += __shfl_xor(s5[tj][o], 16);
          s5[tj][o] += __shfl_xor(s5[tj][o], 32);
        }
        if (q == 0) {
#pragma unroll
          for (int o = 0; o < NOUT; ++o) red[(w * FR + 16 * tj + c16) * NOUT + o] = s5[tj][o];
        }
      }
      __syncthreads();
      if (tid < FR) {
        const long long i = row0 + tid;
        if (i < n) {
#pragma unroll
          for (int o = 0; o < NOUT; ++o)
            yout[i * NOUT + o] = P[OFF_B5 + o] + ((red[(0 * FR + tid) * NOUT + o] + red[(1 * FR + tid) * NOUT + o]) +
                                                  (red[(2 * FR + tid) * NOUT + o] + red[(3 * FR + tid) * NOUT + o]));
        }
      }
    }
  }
}

// The training forward: the network of k_mlp_fused on a batch of n rows,
// R rows per block, keeping what the backward pass reads (TrainSink), with
// the loss and its output gradient in place of the outputs.
constexpr int TR = 64;  // rows per block
__global__ void __launch_bounds__(256, 2) k_mlp_train_fwd(const float *__restrict__ x6, long long ld, int n,
                                                          const float *__restrict__ P, const bf16 *__restrict__ Wt,
                                                          const float *__restrict__ sc, JobP jp, TrainSink ts) {
  constexpr int R = TR;
  constexpr int NT = R / 16;  // row tiles of 16
  constexpr int ZLD = 64 + 4;  // padded rows of the pre-activation staging tiles
  __shared__ __attribute__((aligned(16))) bf16 act[R * ALD];
  __shared__ float xn[R * NIN];
  __shared__ __attribute__((aligned(16))) float zs[4 * 16 * ZLD];  // one 16 x 64 tile per wave
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const long long row0 = (long long)blockIdx.x * R;
  if (row0 >= n) return;
  // standardized input features of the tile (rows past n read as zeros)
  if (tid < R) {
    const long long i = row0 + tid;
    float f[NIN] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < n) {
      features(x6, ld, i, jp, f);
#pragma unroll
      for (int k = 0; k < NIN; ++k) f[k] = (f[k] - sc[S_INOFF + k]) * sc[S_INSCALE + k];
#pragma unroll
      for (int k = 0; k < NIN; ++k) ts.xf[i * NIN + k] = f[k];
    }
#pragma unroll
    for (int k = 0; k < NIN; ++k) xn[tid * NIN + k] = f[k];
  }
  __syncthreads();
  {  // layer 1 (FP32): thread = pair of hidden units x half of the rows
    const int u = 2 * (tid & 127), rb = (tid >> 7) * (R / 2);
    float w0[NIN], w1[NIN];
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      w0[k] = P[OFF_W1 + k * HID + u];
      w1[k] = P[OFF_W1 + k * HID + u + 1];
    }
    const float b0 = P[OFF_B1 + u], b1 = P[OFF_B1 + u + 1];
    for (int r = rb; r < rb + R / 2; ++r) {
      float z0 = b0, z1 = b1;
#pragma unroll
      for (int k = 0; k < NIN; ++k) {
        z0 = fmaf(xn[r * NIN + k], w0[k], z0);
        z1 = fmaf(xn[r * NIN + k], w1[k], z1);
      }
      bf16x2 pr;
      pr[0] = (bf16)silu_f(z0);
      pr[1] = (bf16)silu_f(z1);
      *reinterpret_cast<bf16x2 *>(&act[r * ALD + u]) = pr;
      if (row0 + r < n) *reinterpret_cast<float2 *>(&ts.z[0][(row0 + r) * HID + u]) = float2{z0, z1};
    }
  }
  __syncthreads();
  store_act_tile_t<R>(act, ts.aT[0], ts.ldT, row0, n, tid);
  const int q = lane >> 4, c16 = lane & 15, ub = 64 * w;
  const long long offb[3] = {OFF_B2, OFF_B3, OFF_B4};
  f32x4 acc[4][NT];  // [unit tile][row tile]
  for (int l = 0; l < 3; ++l) {
    const bf16 *W = Wt + (long long)l * HID * HID;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) acc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int k0 = 0; k0 < HID; k0 += 32) {
      bf16x8 aop[4];
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
        aop[ti] = *reinterpret_cast<const bf16x8 *>(W + (ub + 16 * ti + c16) * HID + k0 + 8 * q);
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        const bf16x8 bop = *reinterpret_cast<const bf16x8 *>(&act[(16 * tj + c16) * ALD + k0 + 8 * q]);
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[ti], bop, acc[ti][tj], 0, 0, 0);
      }
    }
    __syncthreads();  // every wave has read the layer's input tile
    {
      // the pre-activations z = acc + bias of this layer: each 16-row tile
      // of the wave's 64 units goes through the wave's own LDS tile, so
      // that a store instruction writes 4 rows x 256 contiguous bytes
      // (whole lines) instead of 16 rows x 64 bytes. One wave writes and
      // reads its tile; its LDS operations complete in order, and the wave
      // barrier keeps the compiler from moving them across each other.
      float *zl = ts.z[l + 1] + row0 * HID;  // the block's rows (32-bit offsets from here)
      float *zw = zs + w * 16 * ZLD;
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
#pragma unroll
        for (int ti = 0; ti < 4; ++ti) {
          const float4 bb = *reinterpret_cast<const float4 *>(&P[offb[l] + ub + 16 * ti + 4 * q]);
          *reinterpret_cast<float4 *>(&zw[c16 * ZLD + 16 * ti + 4 * q]) =
              float4{acc[ti][tj][0] + bb.x, acc[ti][tj][1] + bb.y, acc[ti][tj][2] + bb.z, acc[ti][tj][3] + bb.w};
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int rl = 4 * rr + (lane >> 4), r = 16 * tj + rl;
          const float4 v = *reinterpret_cast<const float4 *>(&zw[rl * ZLD + 4 * c16]);
          if (row0 + r < n) *reinterpret_cast<float4 *>(&zl[r * HID + ub + 4 * c16]) = v;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (l < 2) {
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) {
        const int u0 = ub + 16 * ti + 4 * q;  // this lane's 4 consecutive units
        float bias[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) bias[r] = P[offb[l] + u0 + r];
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
          bf16x4 pk;
#pragma unroll
          for (int r = 0; r < 4; ++r) pk[r] = (bf16)silu_f(acc[ti][tj][r] + bias[r]);
          *reinterpret_cast<bf16x4 *>(&act[(16 * tj + c16) * ALD + u0]) = pk;
        }
      }
      __syncthreads();
      store_act_tile_t<R>(act, ts.aT[l + 1], ts.ldT, row0, n, tid);
    } else {
      // layer 5 (FP32) on a4 = silu(z4): partial sums over this lane's 16
      // units for each of its 8 rows, then over the 4 lane groups
      float s5[NT][NOUT];
#pragma unroll
      for (int tj = 0; tj < NT; ++tj)
#pragma unroll
        for (int o = 0; o < NOUT; ++o) s5[tj][o] = 0.0f;
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) {
        const int u0 = ub + 16 * ti + 4 * q;
        float bias[4], w5[4][NOUT];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          bias[r] = P[offb[l] + u0 + r];
#pragma unroll
          for (int o = 0; o < NOUT; ++o) w5[r][o] = P[OFF_W5 + (u0 + r) * NOUT + o];
        }
#pragma unroll
        for (int tj = 0; tj < NT; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float a4 = silu_f(acc[ti][tj][r] + bias[r]);
#pragma unroll
            for (int o = 0; o < NOUT; ++o) s5[tj][o] = fmaf(a4, w5[r][o], s5[tj][o]);
          }
      }
      float *red = reinterpret_cast<float *>(act);  // [4 waves][R][NOUT]
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
          s5[tj][o] += __shfl_xor(s5[tj][o], 16);
          s5[tj][o] += __shfl_xor(s5[tj][o], 32);
        }
        if (q == 0) {
#pragma unroll
          for (int o = 0; o < NOUT; ++o) red[(w * R + 16 * tj + c16) * NOUT + o] = s5[tj][o];
        }
      }
      __syncthreads();
      float lrow = 0.0f;
      if (tid < R) {
        const long long i = row0 + tid;
        if (i < n) {
#pragma unroll
          for (int o = 0; o < NOUT; ++o) {
            const float y = P[OFF_B5 + o] + ((red[(0 * R + tid) * NOUT + o] + red[(1 * R + tid) * NOUT + o]) +
                                             (red[(2 * R + tid) * NOUT + o] + red[(3 * R + tid) * NOUT + o]));
            {
              // the loss term and its gradient (see TrainSink)
              const float wr = ts.w ? ts.w[i] : 1.0f;
              float g = 0.f;
              if (wr != 0.0f) {
                const float tn = (ts.t[o * ts.ldt + i] - sc[S_OMEAN + o]) / sc[S_OSTD + o];
                const float d = y - tn;
                if (ts.huber > 0.0f && fabsf(d) > ts.huber) {
                  lrow += wr * (2.0f * ts.huber * fabsf(d) - ts.huber * ts.huber);
                  g = 2.0f * wr * copysignf(ts.huber, d);
                } else {
                  lrow += wr * d * d;
                  g = 2.0f * wr * d;
                }
              }
              ts.dy[i * NOUT + o] = g / (float)n;
            }
          }
        }
      }
      {
        // block sum of the loss terms (rows of the first R / 64 waves)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lrow += __shfl_xor(lrow, off);
        if (lane == 0 && w < R / 64) atomicAdd(ts.loss, lrow / (float)n);
      }
    }
  }
}

// error of the decoded prediction against the exact exit, per trust-map cell:
// err = max(|x - x_exact| / b, angle(d, d_exact)); a ray the exact
// integrator did not carry to an exit (absorbed, reflected, ...) makes its
// cell untrusted. The cap job counts only the rows its gate would offer the
// network (heading for a cap, u < 1) and whose prediction is a usable cap
// exit (decode_cap with the gate's margin): the gate rejects the
// others whatever their cell, so they neither count towards nor fail it.
__global__ void __launch_bounds__(256) k_calib(const float *__restrict__ x6, long long ld, int n,
                                               const float *__restrict__ y, const float *__restrict__ sc,
                                               const float *__restrict__ ye, const int *__restrict__ st,
                                               const float *__restrict__ hres, float unresolved, bool infinite,
                                               JobP jp, float margin, unsigned int *__restrict__ cmax,
                                               unsigned int *__restrict__ ccnt) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float phi = x6[i], z = x6[ld + i], al = x6[2 * ld + i], be = x6[3 * ld + i];
  const float pol = x6[4 * ld + i], axis = x6[5 * ld + i];
  if (!entry_ok(phi, z, al, be, pol, axis)) return;
  // an exit the integrator did not resolve is no reference: a drifted
  // Hamiltonian, or total internal reflection at the exit of a side entry
  // into the infinite cylinder (impossible in exact arithmetic: the
  // tangential wave numbers the ray entered with are conserved, so the exit
  // refraction transmits; only drift beyond a grazing entry's normal wave
  // number turns it evanescent)
  if (hres && st[i] == RT_RAY_EXITED && !(hres[i] <= unresolved)) return;
  if (hres && infinite && st[i] == RT_RAY_TIR) return;
  const int kind = kind_of(pol, axis);
  const float b = jp.b;
  int cell;
  float out[NOUT];
  bool usable = true;
  if (jp.job == RT_SUR_CAP) {
    if (!(z >= jp.z0 && z <= jp.z1)) return;
    const float u = cap_fraction(z, al, be, kind, jp);
    if (!(u < 1.0f)) return;
    cell = cell_cap(kind, al, be, u);
    usable = decode_cap(y + i * NOUT, sc, phi, z, al, be, kind, jp, margin, out);
  } else {
    cell = cell_of(kind, al, be);
    decode(y + i * NOUT, sc, phi, z, al, be, kind, jp.a, b, out);
  }
  float err = INFINITY;
  if (st[i] == RT_RAY_EXITED) {
    if (!usable) return;
    float ex[NOUT], xp[3], dp[3], xe[3], de[3];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) ex[o] = ye[o * ld + i];
    exit_ray(out, b, xp, dp);
    exit_ray(ex, b, xe, de);
    float ex2 = 0.f, dd2 = 0.f;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      ex2 += (xp[j] - xe[j]) * (xp[j] - xe[j]);
      dd2 += (dp[j] - de[j]) * (dp[j] - de[j]);
    }
    const float dang = 2.0f * asinf(fminf(1.0f, 0.5f * sqrtf(dd2)));
    err = fmaxf(sqrtf(ex2) / b, dang);
    if (!isfinite(err)) err = INFINITY;
  }
  atomicMax(&cmax[cell], __float_as_uint(err));  // err >= 0: uint order = float order
  atomicAdd(&ccnt[cell], 1u);
}

unsigned int gblocks(long long n, int b) { return (unsigned int)std::max(1LL, (n + b - 1) / b); }

}  // namespace sg

using namespace sg;

struct rt_model_s {
  int device = -1;
  void *base = nullptr;
  float *P = nullptr, *G = nullptr, *m = nullptr, *v = nullptr;  // FP32 [NPARAM]
  bf16 *Pb = nullptr;                                            // BF16 W2..W4
  float *scal = nullptr;                                         // [NSCAL]
  unsigned char *map = nullptr;                                  // trust map [NCELLS]
  unsigned int *cal = nullptr;                                   // calibration max/count [2 * NCELLS]
  double *mom = nullptr;                                         // moments [NMOM]
  float h_scal[NSCAL] = {0};
  std::vector<unsigned char> h_map;
  int map_valid = 0;
  int job = RT_SUR_SIDE;
  float geo[4] = {0.f, 0.f, 0.f, 0.f};  // cap job: r1, r2, z0, z1 of the cloak it was set up for
  rt_model next = nullptr;              // rt_surrogate_chain: rows this model rejects go to next
  rt_model prev = nullptr;              // the model whose rejected rows come here
  rt_gate_opts gate{};
  long long step = 0;
  // activations for up to `cap` rows
  long long cap = 0;
  void *act = nullptr;
  float *z[4] = {nullptr, nullptr, nullptr, nullptr};  // hidden pre-activations (FP32)
  bf16 *aT[3] = {nullptr, nullptr, nullptr};           // a1..a3 (BF16), transposed [256][ldT]
  long long ldT = 0;                                   // row stride of the transposed arrays
  float *p5 = nullptr;                                 // layer-5 gradient partials [L5_MAXB][L5_LD]
  float *dy = nullptr;                                 // [cap][5]
  bf16 *dzb[2] = {nullptr, nullptr};                   // BF16 dz [cap][256], ping-pong
  bf16 *dzT[2] = {nullptr, nullptr};                   // their transposes [256][ldT]
  float *xf = nullptr;                                 // standardized input features [cap][6]
  float *wpart = nullptr;                              // split-K partial weight gradients [64][256 * 256]
  float *cpart = nullptr;                              // per-row-tile column-sum partials [cap / 64][7][256]
  // standardized outputs of the fused inference kernel, and the compacted
  // entry list of the gated inference
  long long ycap = 0;
  float *yinf = nullptr;
  int *idx = nullptr;
  unsigned int *count = nullptr;
};

namespace {

int reserve_acts(rt_model mo, long long n) {
  if (n <= mo->cap) return RT_OK;
  if (mo->act) {
    (void)hipDeviceSynchronize();
    (void)hipFree(mo->act);
    mo->act = nullptr;
    mo->cap = 0;
  }
  const long long cap = std::max(n, 4096LL);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const long long ldT = (cap + 63) & ~63LL;
  const size_t zb = al(sizeof(float) * cap * HID), ab = al(sizeof(bf16) * ldT * HID);
  const size_t yb = al(sizeof(float) * cap * NOUT), fb = al(sizeof(float) * cap * NIN);
  const size_t pb = al(sizeof(float) * L5_MAXB * L5_LD);
  const size_t wb = al(sizeof(float) * 64 * HID * HID), cb = al(sizeof(float) * ((cap + 63) / 64) * (NIN + 1) * HID);
  const size_t bytes = 4 * zb + 3 * ab + yb + 4 * ab + fb + pb + wb + cb;
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RT_E_NOMEM, "hipMalloc of %zu bytes for activations failed", bytes);
  }
  char *c = (char *)p;
  size_t off = 0;
  for (int l = 0; l < 4; ++l) { mo->z[l] = (float *)(c + off); off += zb; }
  for (int l = 0; l < 3; ++l) { mo->aT[l] = (bf16 *)(c + off); off += ab; }
  mo->ldT = ldT;
  mo->dy = (float *)(c + off); off += yb;
  mo->dzb[0] = (bf16 *)(c + off); off += ab;
  mo->dzb[1] = (bf16 *)(c + off); off += ab;
  mo->dzT[0] = (bf16 *)(c + off); off += ab;
  mo->dzT[1] = (bf16 *)(c + off); off += ab;
  mo->xf = (float *)(c + off); off += fb;
  mo->p5 = (float *)(c + off); off += pb;
  mo->wpart = (float *)(c + off); off += wb;
  mo->cpart = (float *)(c + off); off += cb;
  mo->act = p;
  mo->cap = cap;
  return RT_OK;
}

int reserve_yinf(rt_model mo, long long n) {
  if (n <= mo->ycap) return RT_OK;
  if (mo->yinf) {
    (void)hipDeviceSynchronize();
    (void)hipFree(mo->yinf);
    mo->yinf = nullptr;
    mo->ycap = 0;
  }
  const long long cap = std::max(n, 4096LL);
  const size_t yb = (sizeof(float) * cap * NOUT + 255) & ~(size_t)255;
  if (hipMalloc((void **)&mo->yinf, yb + sizeof(int) * cap + 256) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RT_E_NOMEM, "hipMalloc for %lld inference outputs failed", cap);
  }
  mo->idx = (int *)((char *)mo->yinf + yb);
  mo->count = (unsigned int *)((char *)mo->idx + ((sizeof(int) * cap + 255) & ~(size_t)255));
  mo->ycap = cap;
  return RT_OK;
}

// The job parameters of a model's kernels: the cap job carries the
// geometry it was set up for; the side job's features need none, and its
// decoding takes the radii of the cloak description d (if given).
JobP job_for(rt_model mo, const rt_cloak_desc *d) {
  if (mo->job == RT_SUR_CAP) return JobP{RT_SUR_CAP, mo->geo[0], mo->geo[1], mo->geo[2], mo->geo[3]};
  if (!d) return JobP{RT_SUR_SIDE, 0.0f, 0.0f, 0.0f, 0.0f};
  return JobP{RT_SUR_SIDE, (float)d->r1, (float)d->r2, std::isfinite(d->z0) ? (float)d->z0 : -INFINITY,
              std::isfinite(d->z1) ? (float)d->z1 : INFINITY};
}

// standardized outputs of n rows into mo->yinf (fused kernel)
void infer_outputs(rt_model mo, const float *x, long long ld, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_fused, dim3(gblocks(n, FR)), dim3(256), 0, s, x, ld, n, nullptr, nullptr, mo->P, mo->Pb,
                     mo->scal, job_for(mo, nullptr), mo->yinf);
}

// returns the number of K splits used (EPI_SPLIT writes that many partials)
int gemm(hipStream_t s, const bf16 *A, long long lda, const bf16 *B, long long ldb, int M, int N, int K, int epi,
         const float *Z, long long ldz, float *Cf, long long ldcf, bf16 *Cb, long long ldcb, int splits = 1,
         float *colsum = nullptr, bf16 *Cbt = nullptr, long long ldcbt = 0, const float *xf = nullptr) {
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + GK - 1) / GK * GK;  // splits start on a K step
  splits = (K + kchunk - 1) / kchunk;
  const int nct = (int)gblocks(N, GT), nrt = (int)gblocks(M, GT);
  const bool veca = lda % 8 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0;
  const bool vecb = ldb % 8 == 0 && reinterpret_cast<uintptr_t>(B) % 16 == 0;
  Gemm g{A, lda, B, ldb, veca, vecb, M, N, K, kchunk, epi, nct, nrt, Z, ldz, Cf, ldcf, Cb, ldcb, colsum, xf, Cbt, ldcbt};
  // 64 x 64 block tiles: 128 x 128 ones measured slower on the training
  // shapes, whose time goes to the epilogue's activation traffic rather than
  // to the MFMAs
  hipLaunchKernelGGL(k_gemm, dim3((unsigned)((long long)nct * nrt * splits)), dim3(256), 0, s, g);
  return splits;
}

// BF16 weights of W2 (l = 0), W3 (1), W4 (2): transposed [out][in] and row-major [in][out]
const bf16 *wb(rt_model mo, int l) { return mo->Pb + (long long)l * HID * HID; }
const bf16 *wr(rt_model mo, int l) { return mo->Pb + NBF + (long long)l * HID * HID; }

int split_for(int n) { return std::min(64, std::max(1, n / 512)); }

// training forward of n rows (the fused network, keeping xf, z1..z4 and
// a1..a3 for the backward pass) with the loss and its output gradient dy;
// then the gradients of that loss into mo->G, the loss into scal[S_LOSS]
void forward_backward(rt_model mo, const float *x, const float *t, long long ld, const float *wrow, int n,
                      float huber, hipStream_t s) {
  float *loss = mo->scal + S_LOSS;
  hipLaunchKernelGGL(k_fill, dim3(gblocks(NPARAM, 256)), dim3(256), 0, s, mo->G, NPARAM, 0.0f);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, loss, 1LL, 0.0f);
  const long long ldT = mo->ldT;
  TrainSink ts{mo->xf, {mo->z[0], mo->z[1], mo->z[2], mo->z[3]}, {mo->aT[0], mo->aT[1], mo->aT[2]}, ldT, t, ld,
               wrow, huber, mo->dy, loss};
  hipLaunchKernelGGL(k_mlp_train_fwd, dim3(gblocks(n, TR)), dim3(256), 0, s, x, ld, n, mo->P, mo->Pb, mo->scal,
                     job_for(mo, nullptr), ts);
  // layer 5: its per-element work (dz of layer 4) is as large as a hidden
  // layer's and parallel over rows: one block per 64 rows, up to 1024
  // blocks; the blocks' partial sums of the layer-5 weights and biases and
  // of b4 are added in a second pass
  const int l5_grid = std::min(L5_MAXB, (int)gblocks(n, 64));
  hipLaunchKernelGGL(k_layer5_back, dim3(l5_grid), dim3(HID), 0, s, mo->dy, mo->z[3], n, mo->P, mo->p5, mo->dzb[1],
                     mo->dzT[1], ldT);
  hipLaunchKernelGGL(k_sum_rows, dim3((L5_N + 63) / 64, std::max(1, std::min(16, l5_grid / 4))), dim3(256), 0, s,
                     mo->p5, l5_grid, (long long)L5_LD, L5_N, mo->G + OFF_B4);
  // hidden layers from the top: dz of layer l + 1 in dzb[cur] (BF16,
  // row-major) and dzT[cur] (its transpose)
  const long long offw[3] = {OFF_W2, OFF_W3, OFF_W4}, offb[3] = {OFF_B2, OFF_B3, OFF_B4};
  int cur = 1;
  for (int l = 3; l >= 1; --l) {
    // dW_{l+1} = a_l^T dz: both operands transposed so that the batch (the
    // sum) is their contiguous index, split over the rows into partial
    // products, then summed
    const int splits = gemm(s, mo->aT[l - 1], ldT, mo->dzT[cur], ldT, HID, HID, n, EPI_SPLIT, nullptr, 0,
                            mo->wpart, HID, nullptr, 0, split_for(n));
    hipLaunchKernelGGL(k_sum_rows, dim3(HID * HID / 64, 1), dim3(256), 0, s, mo->wpart, splits,
                       (long long)HID * HID, HID * HID, mo->G + offw[l - 1]);
    // dz_l = (dz W_{l+1}^T) * silu'(z_l) (B(k, j) = W(in=j, out=k), row-major
    // copy) with its per-row-tile column sums: for l >= 2 dz_l goes out in
    // BF16 (both layouts) and the sums make db_l; dz_1 (FP32) never leaves
    // the tile: its sums xf^T dz_1 and sum dz_1 are the gradients of W1 and
    // b1 (contiguous in the parameter vector)
    const int nrt = (int)gblocks(n, 64), ns = l >= 2 ? 1 : NIN + 1;
    gemm(s, mo->dzb[cur], HID, wr(mo, l - 1), HID, n, HID, HID, EPI_DSILU, mo->z[l - 1], HID, nullptr, 0,
         l >= 2 ? mo->dzb[cur ^ 1] : nullptr, HID, 1, mo->cpart, l >= 2 ? mo->dzT[cur ^ 1] : nullptr, ldT,
         l >= 2 ? nullptr : mo->xf);
    hipLaunchKernelGGL(k_sum_rows, dim3(ns * HID / 64, std::max(1, std::min(16, nrt / 4))), dim3(256), 0, s,
                       mo->cpart, nrt, (long long)ns * HID, ns * HID, mo->G + (l >= 2 ? offb[l - 2] : OFF_W1));
    cur ^= 1;
  }
}

int check_model(rt_model mo) {
  if (!mo || !mo->P) return fail(RT_E_INVALID, "model is NULL");
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != mo->device) return fail(RT_E_INVALID, "model was created on device %d, current is %d", mo->device, dev);
  return RT_OK;
}

int check_rows(long long n, long long ld, const void *x6) {
  if (n < 1 || n > (1LL << 24)) return fail(RT_E_INVALID, "n must be in [1, 2^24]");
  if (ld < n) return fail(RT_E_INVALID, "ld must be >= n");
  if (!x6) return fail(RT_E_INVALID, "x6 is required");
  return RT_OK;
}

int upload_scal(rt_model mo) {
  if (hipMemcpy(mo->scal, mo->h_scal, sizeof(float) * S_LOSS, hipMemcpyHostToDevice) != hipSuccess)
    return fail(RT_E_DEVICE, "copy of the scaling failed");
  return RT_OK;
}

int upload_map(rt_model mo) {
  if (hipMemcpy(mo->map, mo->h_map.data(), NCELLS, hipMemcpyHostToDevice) != hipSuccess)
    return fail(RT_E_DEVICE, "copy of the trust map failed");
  return RT_OK;
}

int cloak_geometry(const rt_cloak *cloaks, int32_t n_cloaks, rt_cloak_desc &d) {
  if (n_cloaks < 1 || n_cloaks > 2 || !cloaks || !cloaks[0]) return fail(RT_E_INVALID, "need 1 or 2 cloak handles");
  if (rt_cloak_get_desc(cloaks[0], &d) != RT_OK) return fail(RT_E_INVALID, "bad cloak handle");
  return RT_OK;
}

int launch_err(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return RT_OK;
}

// A cap model works on cloaks of the geometry it was set up for.
int check_geometry(rt_model mo, const rt_cloak_desc &d) {
  if (mo->job != RT_SUR_CAP) return RT_OK;
  if ((float)d.r1 != mo->geo[0] || (float)d.r2 != mo->geo[1] || (float)d.z0 != mo->geo[2] ||
      (float)d.z1 != mo->geo[3])
    return fail(RT_E_INVALID, "the cloaks' geometry (r1 %g, r2 %g, z %g..%g) is not the one the cap model was set "
                              "up for (r1 %g, r2 %g, z %g..%g)", d.r1, d.r2, d.z0, d.z1, mo->geo[0], mo->geo[1],
                mo->geo[2], mo->geo[3]);
  return RT_OK;
}

}  // namespace

int surrogate_check_ready(rt_model mo) {
  for (rt_model m = mo; m; m = m == mo ? mo->next : nullptr) {
    int e = check_model(m);
    if (e) return e;
    if (!m->map_valid)
      return fail(RT_E_INVALID, "the %smodel has no calibrated trust map (rt_surrogate_calibrate)",
                  m == mo ? "" : "chained ");
  }
  return RT_OK;
}

double surrogate_exit_tolerance(rt_model mo) {
  return mo->next ? std::max(mo->gate.tol, mo->next->gate.tol) : mo->gate.tol;
}

int surrogate_predict_gated(rt_model mo, const rt_cloak_desc &d, int64_t n, int64_t ld, const float *x6, float *y5,
                            uint8_t *fallback, int32_t *status, hipStream_t s) {
  int e = surrogate_check_ready(mo);
  if (!e) e = check_geometry(mo, d);
  if (!e && mo->next) e = check_geometry(mo->next, d);
  if (e) return e;
  if (n == 0) return RT_OK;
  if (n < 0 || ld < n || !x6 || !y5 || !fallback || !status)
    return fail(RT_E_INVALID, "bad rows for the surrogate (n, ld or a NULL array)");
  const long long batch = std::min<long long>(n, 1LL << 24);
  // the model, then the chained one on the rows the first rejected
  for (rt_model m = mo; m; m = m == mo ? mo->next : nullptr) {
    GateP gp;
    gp.a = (float)d.r1;
    gp.b = (float)d.r2;
    gp.z0 = std::isfinite(d.z0) ? (float)d.z0 : -INFINITY;
    gp.z1 = std::isfinite(d.z1) ? (float)d.z1 : INFINITY;
    gp.hres_max = (float)m->gate.hres_max;
    gp.cap_margin = (float)m->gate.cap_margin;
    gp.p_min = (float)m->gate.p_min;
    const JobP jp = job_for(m, &d);
    e = reserve_yinf(m, batch);
    if (e) return e;
    for (long long off = 0; off < n; off += batch) {
      const int rows = (int)std::min<long long>(batch, n - off);
      const float *x = x6 + off;
      // entries that pass the input gate only go through the network
      // (compacted), then the output half of the gate
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, m->count, 1LL);
      hipLaunchKernelGGL(k_pregate, dim3(gblocks(rows, 256)), dim3(256), 0, s, x, (long long)ld, rows, m->map, gp, jp,
                         m == mo ? 0 : 1, fallback + off, m->idx, m->count);
      hipLaunchKernelGGL(k_mlp_fused, dim3(gblocks(rows, FR)), dim3(256), 0, s, x, (long long)ld, rows, m->idx,
                         m->count, m->P, m->Pb, m->scal, jp, m->yinf);
      hipLaunchKernelGGL(k_gate_idx, dim3(gblocks(rows, 256)), dim3(256), 0, s, x, (long long)ld, m->idx, m->count,
                         m->yinf, m->scal, m->map, gp, jp, y5 + off, fallback + off, status + off);
    }
  }
  return launch_err("surrogate launch");
}

extern "C" {

int rt_surrogate_create(uint64_t seed, rt_model *out) {
  if (!out) return fail(RT_E_INVALID, "out is NULL");
  *out = nullptr;
  rt_model mo = new (std::nothrow) rt_model_s;
  if (!mo) return fail(RT_E_NOMEM, "host allocation failed");
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t pb = al(sizeof(float) * NPARAM), bb = al(sizeof(bf16) * 2 * NBF), sb = al(sizeof(float) * NSCAL),
               mb = al(NCELLS), cb = al(sizeof(unsigned int) * 2 * NCELLS), ob = al(sizeof(double) * NMOM);
  const size_t bytes = 4 * pb + bb + sb + mb + cb + ob;
  if (hipMalloc(&mo->base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete mo;
    return fail(RT_E_NOMEM, "hipMalloc of the model failed");
  }
  (void)hipGetDevice(&mo->device);
  char *c = (char *)mo->base;
  size_t off = 0;
  mo->P = (float *)(c + off); off += pb;
  mo->G = (float *)(c + off); off += pb;
  mo->m = (float *)(c + off); off += pb;
  mo->v = (float *)(c + off); off += pb;
  mo->Pb = (bf16 *)(c + off); off += bb;
  mo->scal = (float *)(c + off); off += sb;
  mo->map = (unsigned char *)(c + off); off += mb;
  mo->cal = (unsigned int *)(c + off); off += cb;
  mo->mom = (double *)(c + off); off += ob;
  // weights and biases uniform in +-1/sqrt(fan_in) from a seeded Mersenne
  // twister, drawn layer by layer (weights row-major, then biases)
  std::vector<float> h(NPARAM, 0.0f);
  std::mt19937_64 rng(seed);
  const int fan_in[5] = {NIN, HID, HID, HID, HID}, fan_out[5] = {HID, HID, HID, HID, NOUT};
  const long long offw[5] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4, OFF_W5};
  const long long offb[5] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4, OFF_B5};
  for (int l = 0; l < 5; ++l) {
    const float k = 1.0f / std::sqrt((float)fan_in[l]);
    std::uniform_real_distribution<float> U(-k, k);
    for (long long e = 0; e < (long long)fan_in[l] * fan_out[l]; ++e) h[offw[l] + e] = U(rng);
    for (int j = 0; j < fan_out[l]; ++j) h[offb[l] + j] = U(rng);
  }
  for (int k = 0; k < NIN; ++k) { mo->h_scal[S_INOFF + k] = 0.0f; mo->h_scal[S_INSCALE + k] = 1.0f; }
  for (int o = 0; o < NOUT; ++o) { mo->h_scal[S_OMEAN + o] = 0.0f; mo->h_scal[S_OSTD + o] = 1.0f; }
  mo->h_map.assign(NCELLS, 0);
  mo->gate.tol = 1e-3;
  mo->gate.hres_max = 1e-4;
  mo->gate.cap_margin = 1e-2;
  mo->gate.min_count = 8;
  mo->gate.p_min = 1e-4;
  bool ok = hipMemcpy(mo->P, h.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice) == hipSuccess &&
            upload_scal(mo) == RT_OK && upload_map(mo) == RT_OK;
  if (ok) {
    hipLaunchKernelGGL(k_fill, dim3(gblocks(NPARAM, 256)), dim3(256), 0, 0, mo->m, NPARAM, 0.0f);
    hipLaunchKernelGGL(k_fill, dim3(gblocks(NPARAM, 256)), dim3(256), 0, 0, mo->v, NPARAM, 0.0f);
    hipLaunchKernelGGL(k_refresh_bf16, dim3(gblocks(NPARAM, 256)), dim3(256), 0, 0, mo->P, mo->Pb);
    ok = hipDeviceSynchronize() == hipSuccess;
  }
  if (!ok) {
    (void)hipFree(mo->base);
    delete mo;
    return fail(RT_E_DEVICE, "model initialization failed");
  }
  *out = mo;
  return RT_OK;
}

int rt_surrogate_free(rt_model mo) {
  if (!mo) return RT_OK;
  (void)hipDeviceSynchronize();
  if (mo->prev) mo->prev->next = nullptr;
  if (mo->next) mo->next->prev = nullptr;
  if (mo->act) (void)hipFree(mo->act);
  if (mo->yinf) (void)hipFree(mo->yinf);
  if (mo->base) (void)hipFree(mo->base);
  delete mo;
  return RT_OK;
}

int rt_surrogate_nparams(int64_t *count) {
  if (!count) return fail(RT_E_INVALID, "count is NULL");
  *count = NPARAM;
  return RT_OK;
}

int rt_surrogate_get_params(rt_model mo, float *host) {
  int e = check_model(mo);
  if (e) return e;
  if (!host) return fail(RT_E_INVALID, "host is NULL");
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(host, mo->P, sizeof(float) * NPARAM, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(RT_E_DEVICE, "copy failed");
  return RT_OK;
}

int rt_surrogate_set_params(rt_model mo, const float *host) {
  int e = check_model(mo);
  if (e) return e;
  if (!host) return fail(RT_E_INVALID, "host is NULL");
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(mo->P, host, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess)
    return fail(RT_E_DEVICE, "copy failed");
  hipLaunchKernelGGL(k_refresh_bf16, dim3(gblocks(NPARAM, 256)), dim3(256), 0, 0, mo->P, mo->Pb);
  hipLaunchKernelGGL(k_fill, dim3(gblocks(NPARAM, 256)), dim3(256), 0, 0, mo->m, NPARAM, 0.0f);
  hipLaunchKernelGGL(k_fill, dim3(gblocks(NPARAM, 256)), dim3(256), 0, 0, mo->v, NPARAM, 0.0f);
  if (hipDeviceSynchronize() != hipSuccess) return fail(RT_E_DEVICE, "refresh failed");
  mo->step = 0;
  return RT_OK;
}

int rt_surrogate_get_scaling(rt_model mo, float *scaling22) {
  int e = check_model(mo);
  if (e) return e;
  if (!scaling22) return fail(RT_E_INVALID, "scaling is NULL");
  memcpy(scaling22, mo->h_scal, sizeof(float) * S_LOSS);
  return RT_OK;
}

int rt_surrogate_set_scaling(rt_model mo, const float *scaling22) {
  int e = check_model(mo);
  if (e) return e;
  if (!scaling22) return fail(RT_E_INVALID, "scaling is NULL");
  for (int k = 0; k < S_LOSS; ++k)
    if (!std::isfinite(scaling22[k])) return fail(RT_E_INVALID, "scaling values must be finite");
  for (int o = 0; o < NOUT; ++o)
    if (!(scaling22[S_OSTD + o] > 0.0f)) return fail(RT_E_INVALID, "out_std must be > 0");
  memcpy(mo->h_scal, scaling22, sizeof(float) * S_LOSS);
  if (hipDeviceSynchronize() != hipSuccess) return fail(RT_E_DEVICE, "synchronize failed");
  return upload_scal(mo);
}

int rt_surrogate_fit_scaling(rt_model mo, int64_t n, int64_t ld, const float *x6, const float *t5, const float *w,
                             void *stream) {
  int e = check_model(mo);
  if (!e) e = check_rows(n, ld, x6);
  if (e) return e;
  if (!t5) return fail(RT_E_INVALID, "t5 is required");
  hipStream_t s = (hipStream_t)stream;
  double h[NMOM];
  hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, mo->mom, NMOM);
  hipLaunchKernelGGL(k_moments, dim3(std::min(gblocks(n, 256), 1024u)), dim3(256), 0, s, x6, t5, (long long)ld, w,
                     (int)n, job_for(mo, nullptr), mo->mom);
  if (hipMemcpyAsync(h, mo->mom, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(RT_E_DEVICE, "moments failed");
  const double W = h[NMOM - 1];
  if (!(W > 0.0)) return fail(RT_E_INVALID, "no row has a nonzero weight");
  for (int k = 0; k < NIN + NOUT; ++k) {
    const double mean = h[2 * k] / W;
    const double var = std::max(0.0, h[2 * k + 1] / W - mean * mean);
    const double sd = std::sqrt(var);
    if (k < NIN) {
      mo->h_scal[S_INOFF + k] = (float)mean;
      mo->h_scal[S_INSCALE + k] = (float)(1.0 / std::max(sd, 1e-6));
    } else {
      mo->h_scal[S_OMEAN + (k - NIN)] = (float)mean;
      mo->h_scal[S_OSTD + (k - NIN)] = std::max((float)sd, OUT_STD_FLOOR);
    }
  }
  return upload_scal(mo);
}

int grad_impl(rt_model mo, int64_t n, int64_t ld, const float *x6, const float *t5, const float *w, float huber,
              float *grads, float *loss, void *stream);

int rt_surrogate_grad(rt_model mo, int64_t n, int64_t ld, const float *x6, const float *t5, const float *w,
                      float huber, float *grads, float *loss, void *stream) {
  if (!(huber >= 0.0f)) return fail(RT_E_INVALID, "huber must be >= 0");
  return grad_impl(mo, n, ld, x6, t5, w, huber, grads, loss, stream);
}

int grad_impl(rt_model mo, int64_t n, int64_t ld, const float *x6, const float *t5, const float *w, float huber,
              float *grads, float *loss, void *stream) {
  int e = check_model(mo);
  if (!e) e = check_rows(n, ld, x6);
  if (e) return e;
  if (!t5) return fail(RT_E_INVALID, "t5 is required");
  e = reserve_acts(mo, n);
  if (e) return e;
  hipStream_t s = (hipStream_t)stream;
  forward_backward(mo, x6, t5, ld, w, (int)n, huber, s);
  if (grads) (void)hipMemcpyAsync(grads, mo->G, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, s);
  if (loss) (void)hipMemcpyAsync(loss, mo->scal + S_LOSS, sizeof(float), hipMemcpyDeviceToDevice, s);
  return launch_err("gradient launch");
}

int check_train_opts(const rt_train_opts *opts) {
  if (!opts) return fail(RT_E_INVALID, "opts is NULL");
  if (!(opts->lr >= 0.0f) || !(opts->beta1 >= 0.0f && opts->beta1 < 1.0f) ||
      !(opts->beta2 >= 0.0f && opts->beta2 < 1.0f) || !(opts->eps > 0.0f) || !(opts->weight_decay >= 0.0f) ||
      !(opts->huber >= 0.0f))
    return fail(RT_E_INVALID, "need lr >= 0, 0 <= beta1, beta2 < 1, eps > 0, weight_decay >= 0, huber >= 0");
  return RT_OK;
}

// one AdamW step with the gradient G (device, NPARAM floats); advances the
// step count that the bias corrections use
int adamw_step(rt_model mo, const float *G, const rt_train_opts *opts, hipStream_t s) {
  mo->step += 1;
  // bias corrections 1 - beta^t formed in FP64 and rounded once: 1 - beta2^t
  // cancels for early steps (0.039 at beta2 = 0.995, t = 8), and rounding
  // beta2^t to FP32 first would cost it 2^-24 / 0.039 relative
  const float c1 = (float)(1.0 - std::pow((double)opts->beta1, (double)mo->step));
  const float c2 = (float)(1.0 - std::pow((double)opts->beta2, (double)mo->step));
  hipLaunchKernelGGL(k_adamw, dim3(gblocks(NPARAM, 256)), dim3(256), 0, s, mo->P, G, mo->m, mo->v, mo->Pb,
                     opts->lr, opts->weight_decay, opts->beta1, opts->beta2, c1, c2, opts->eps);
  return launch_err("optimizer launch");
}

int rt_surrogate_train(rt_model mo, int64_t n, int64_t ld, const float *x6, const float *t5, const float *w,
                       const rt_train_opts *opts, float *loss, void *stream) {
  int e = check_train_opts(opts);
  if (e) return e;
  e = grad_impl(mo, n, ld, x6, t5, w, opts->huber, nullptr, loss, stream);
  if (e) return e;
  return adamw_step(mo, mo->G, opts, (hipStream_t)stream);
}

int rt_surrogate_step(rt_model mo, const float *grads, const rt_train_opts *opts, void *stream) {
  int e = check_model(mo);
  if (!e) e = check_train_opts(opts);
  if (e) return e;
  if (!grads) return fail(RT_E_INVALID, "grads is NULL");
  return adamw_step(mo, grads, opts, (hipStream_t)stream);
}

int rt_surrogate_get_state(rt_model mo, float *m_host, float *v_host, int64_t *step) {
  int e = check_model(mo);
  if (e) return e;
  if (hipDeviceSynchronize() != hipSuccess) return fail(RT_E_DEVICE, "synchronize failed");
  if ((m_host && hipMemcpy(m_host, mo->m, sizeof(float) * NPARAM, hipMemcpyDeviceToHost) != hipSuccess) ||
      (v_host && hipMemcpy(v_host, mo->v, sizeof(float) * NPARAM, hipMemcpyDeviceToHost) != hipSuccess))
    return fail(RT_E_DEVICE, "copy failed");
  if (step) *step = mo->step;
  return RT_OK;
}

int rt_surrogate_set_state(rt_model mo, const float *m_host, const float *v_host, int64_t step) {
  int e = check_model(mo);
  if (e) return e;
  if (!m_host || !v_host) return fail(RT_E_INVALID, "m and v are required");
  if (step < 0) return fail(RT_E_INVALID, "step must be >= 0");
  for (long long i = 0; i < NPARAM; ++i)
    if (!std::isfinite(m_host[i]) || !(v_host[i] >= 0.0f) || !std::isfinite(v_host[i]))
      return fail(RT_E_INVALID, "moments must be finite and v >= 0 (entry %lld)", i);
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(mo->m, m_host, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(mo->v, v_host, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess)
    return fail(RT_E_DEVICE, "copy failed");
  mo->step = step;
  return RT_OK;
}

int rt_surrogate_forward(rt_model mo, int64_t n, int64_t ld, const float *x6, float *t5, void *stream) {
  int e = check_model(mo);
  if (!e) e = check_rows(n, ld, x6);
  if (e) return e;
  if (!t5) return fail(RT_E_INVALID, "t5 is required");
  e = reserve_yinf(mo, n);
  if (e) return e;
  hipStream_t s = (hipStream_t)stream;
  infer_outputs(mo, x6, ld, (int)n, s);
  hipLaunchKernelGGL(k_destd, dim3(gblocks(n * NOUT, 256)), dim3(256), 0, s, mo->yinf, (int)n, (long long)ld,
                     mo->scal, t5);
  return launch_err("forward launch");
}

int rt_surrogate_encode_job(int32_t job, const rt_cloak *cloaks, int32_t n_cloaks, int64_t n, int64_t ld,
                            const float *x6, const float *y5, const int32_t *status, float *t5, float *w,
                            void *stream) {
  rt_cloak_desc d;
  int e = cloak_geometry(cloaks, n_cloaks, d);
  if (e) return e;
  if (job != RT_SUR_SIDE && job != RT_SUR_CAP) return fail(RT_E_INVALID, "job must be RT_SUR_SIDE or RT_SUR_CAP");
  if (job == RT_SUR_CAP && (!std::isfinite(d.z0) || !std::isfinite(d.z1) || !(d.z1 > d.z0)))
    return fail(RT_E_INVALID, "the cap job needs cloaks of finite height");
  if (n == 0) return RT_OK;
  e = check_rows(n, ld, x6);
  if (e) return e;
  if (!y5 || !status || !t5 || !w) return fail(RT_E_INVALID, "y5, status, t5 and w are required");
  if (job == RT_SUR_CAP) {
    const JobP jp{RT_SUR_CAP, (float)d.r1, (float)d.r2, (float)d.z0, (float)d.z1};
    hipLaunchKernelGGL(k_encode_cap, dim3(gblocks(n, 256)), dim3(256), 0, (hipStream_t)stream, x6, y5, status,
                       (long long)ld, (long long)n, jp, t5, w);
  } else {
    hipLaunchKernelGGL(k_encode, dim3(gblocks(n, 256)), dim3(256), 0, (hipStream_t)stream, x6, y5, status,
                       (long long)ld, (long long)n, (float)d.r1, (float)d.r2, t5, w);
  }
  return launch_err("encode launch");
}

int rt_surrogate_encode(const rt_cloak *cloaks, int32_t n_cloaks, int64_t n, int64_t ld, const float *x6,
                        const float *y5, const int32_t *status, float *t5, float *w, void *stream) {
  return rt_surrogate_encode_job(RT_SUR_SIDE, cloaks, n_cloaks, n, ld, x6, y5, status, t5, w, stream);
}

int rt_surrogate_calibrate(rt_model mo, const rt_cloak *cloaks, int32_t n_cloaks, int64_t n, int64_t ld,
                           const float *x6, const float *y5_exact, const int32_t *status_exact,
                           const float *hres_exact, const rt_gate_opts *gate, double *trusted_fraction,
                           void *stream) {
  int e = check_model(mo);
  if (e) return e;
  rt_cloak_desc d;
  e = cloak_geometry(cloaks, n_cloaks, d);
  if (!e) e = check_geometry(mo, d);
  if (!e) e = check_rows(n, ld, x6);
  if (e) return e;
  if (!y5_exact || !status_exact || !gate) return fail(RT_E_INVALID, "y5_exact, status_exact and gate are required");
  if (!(gate->tol > 0.0) || !(gate->hres_max > 0.0) || !(gate->cap_margin >= 0.0) || gate->min_count < 1 ||
      gate->dilate < 0 || gate->dilate > 8 || (hres_exact && !(gate->unresolved > 0.0)) ||
      !(gate->p_min >= 0.0 && gate->p_min < 1.0))
    return fail(RT_E_INVALID, "gate needs tol > 0, hres_max > 0, cap_margin >= 0, min_count >= 1, "
                              "0 <= dilate <= 8, 0 <= p_min < 1 and, with hres_exact, unresolved > 0");
  e = reserve_yinf(mo, n);
  if (e) return e;
  hipStream_t s = (hipStream_t)stream;
  infer_outputs(mo, x6, ld, (int)n, s);
  hipLaunchKernelGGL(k_fill_u32, dim3(gblocks(2LL * NCELLS, 256)), dim3(256), 0, s, mo->cal, 2LL * NCELLS);
  hipLaunchKernelGGL(k_calib, dim3(gblocks(n, 256)), dim3(256), 0, s, x6, (long long)ld, (int)n, mo->yinf, mo->scal,
                     y5_exact, status_exact, hres_exact, (float)gate->unresolved,
                     !std::isfinite(d.z0) && !std::isfinite(d.z1), job_for(mo, &d), (float)gate->cap_margin, mo->cal,
                     mo->cal + NCELLS);
  std::vector<unsigned int> h(2 * NCELLS);
  if (hipMemcpyAsync(h.data(), mo->cal, sizeof(unsigned int) * 2 * NCELLS, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(RT_E_DEVICE, "calibration failed");
  std::vector<unsigned char> good(NCELLS);
  for (int c = 0; c < NCELLS; ++c) {
    float mx;
    memcpy(&mx, &h[c], sizeof(float));
    good[c] = h[NCELLS + c] >= (unsigned int)gate->min_count && mx <= (float)gate->tol;
  }
  // dilation within each (axis, branch) block over the cell grid's
  // dimensions: (alpha, beta) for the side job, (alpha, |beta|, u) for the
  // cap job
  const int dl = gate->dilate;
  const bool capj = mo->job == RT_SUR_CAP;
  const int na = capj ? CAP_A : NCELL_A, nb = capj ? CAP_B : NCELL_B, nu = capj ? CAP_U : 1;
  const int du = capj ? dl : 0;
  long long trusted = 0;
  for (int k = 0; k < NCOMBO; ++k)
    for (int ia = 0; ia < na; ++ia)
      for (int ib = 0; ib < nb; ++ib)
        for (int iu = 0; iu < nu; ++iu) {
          bool ok = true;
          for (int da = -dl; da <= dl && ok; ++da)
            for (int db = -dl; db <= dl && ok; ++db)
              for (int dv = -du; dv <= du && ok; ++dv) {
                const int ja = ia + da, jb = ib + db, ju = iu + dv;
                if (ja < 0 || ja >= na || jb < 0 || jb >= nb || ju < 0 || ju >= nu) continue;
                ok = good[((k * na + ja) * nb + jb) * nu + ju] != 0;
              }
          mo->h_map[((k * na + ia) * nb + ib) * nu + iu] = ok ? 1 : 0;
          trusted += ok;
        }
  mo->gate = *gate;
  mo->map_valid = 1;
  if (trusted_fraction) *trusted_fraction = (double)trusted / NCELLS;
  return upload_map(mo);
}

int rt_surrogate_get_map(rt_model mo, uint8_t *host, int32_t *cells_alpha, int32_t *cells_beta, int32_t *cells_u) {
  int e = check_model(mo);
  if (e) return e;
  const bool capj = mo->job == RT_SUR_CAP;
  if (cells_alpha) *cells_alpha = capj ? CAP_A : NCELL_A;
  if (cells_beta) *cells_beta = capj ? CAP_B : NCELL_B;
  if (cells_u) *cells_u = capj ? CAP_U : 1;
  if (host) memcpy(host, mo->h_map.data(), NCELLS);
  return RT_OK;
}

int rt_surrogate_set_job(rt_model mo, int32_t job, rt_cloak cloak) {
  int e = check_model(mo);
  if (e) return e;
  if (job != RT_SUR_SIDE && job != RT_SUR_CAP) return fail(RT_E_INVALID, "job must be RT_SUR_SIDE or RT_SUR_CAP");
  float geo[4] = {0.f, 0.f, 0.f, 0.f};
  if (job == RT_SUR_CAP) {
    rt_cloak_desc d;
    if (!cloak || rt_cloak_get_desc(cloak, &d) != RT_OK) return fail(RT_E_INVALID, "the cap job needs a cloak handle");
    if (!std::isfinite(d.z0) || !std::isfinite(d.z1) || !(d.z1 > d.z0))
      return fail(RT_E_INVALID, "the cap job needs a cloak of finite height");
    geo[0] = (float)d.r1;
    geo[1] = (float)d.r2;
    geo[2] = (float)d.z0;
    geo[3] = (float)d.z1;
  }
  mo->job = job;
  memcpy(mo->geo, geo, sizeof(geo));
  // the cells of the trust map change meaning
  std::fill(mo->h_map.begin(), mo->h_map.end(), 0);
  mo->map_valid = 0;
  return upload_map(mo);
}

int rt_surrogate_get_job(rt_model mo, int32_t *job) {
  int e = check_model(mo);
  if (e) return e;
  if (!job) return fail(RT_E_INVALID, "job is NULL");
  *job = mo->job;
  return RT_OK;
}

int rt_surrogate_chain(rt_model first, rt_model next) {
  int e = check_model(first);
  if (e) return e;
  if (next) {
    e = check_model(next);
    if (e) return e;
    if (next == first) return fail(RT_E_INVALID, "a model cannot follow itself");
    if (next->next || first->prev) return fail(RT_E_INVALID, "chains hold two models");
    if (next->prev && next->prev != first) return fail(RT_E_INVALID, "next already follows another model");
  }
  if (first->next) first->next->prev = nullptr;
  first->next = next;
  if (next) next->prev = first;
  return RT_OK;
}

int rt_surrogate_infer(rt_model mo, const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts, int64_t n,
                       int64_t ld, const float *x6, float *y5, uint8_t *fallback, int32_t *status, void *stream) {
  int e = check_model(mo);
  if (e) return e;
  rt_cloak_desc d;
  e = cloak_geometry(cloaks, n_cloaks, d);
  if (e) return e;
  if (!opts) return fail(RT_E_INVALID, "opts is NULL");
  if (n == 0) return RT_OK;
  e = check_rows(n, ld, x6);
  if (e) return e;
  if (!y5 || !fallback || !status) return fail(RT_E_INVALID, "y5, fallback and status are required");
  e = surrogate_predict_gated(mo, d, n, ld, x6, y5, fallback, status, (hipStream_t)stream);
  if (e) return e;
  // the exact integrator traces the rejected rays (one persistent launch)
  return rt_transit_exact(cloaks, n_cloaks, opts, n, ld, x6, fallback, y5, status, nullptr, nullptr, stream);
}

int rt_surrogate_save(rt_model mo, const char *path) {
  int e = check_model(mo);
  if (e) return e;
  if (!path) return fail(RT_E_INVALID, "path is NULL");
  std::vector<float> h(NPARAM);
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(h.data(), mo->P, sizeof(float) * NPARAM, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(RT_E_DEVICE, "copy failed");
  FILE *f = fopen(path, "wb");
  if (!f) return fail(RT_E_INVALID, "cannot open %s", path);
  const char magic[8] = {'R', 'T', 'M', 'L', 'P', '0', '5', '\0'};
  const long long np = NPARAM, nc = NCELLS;
  const int valid = mo->map_valid;
  bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&np, sizeof(np), 1, f) == 1 &&
            fwrite(mo->h_scal, sizeof(float), S_LOSS, f) == (size_t)S_LOSS &&
            fwrite(h.data(), sizeof(float), NPARAM, f) == (size_t)NPARAM && fwrite(&nc, sizeof(nc), 1, f) == 1 &&
            fwrite(&valid, sizeof(valid), 1, f) == 1 && fwrite(&mo->gate, sizeof(mo->gate), 1, f) == 1 &&
            fwrite(mo->h_map.data(), 1, NCELLS, f) == (size_t)NCELLS && fwrite(&mo->job, sizeof(int), 1, f) == 1 &&
            fwrite(mo->geo, sizeof(float), 4, f) == 4;
  ok = (fclose(f) == 0) && ok;
  return ok ? RT_OK : fail(RT_E_INVALID, "write to %s failed", path);
}

int rt_surrogate_load(const char *path, rt_model *out) {
  if (!path || !out) return fail(RT_E_INVALID, "path and out are required");
  *out = nullptr;
  FILE *f = fopen(path, "rb");
  if (!f) return fail(RT_E_INVALID, "cannot open %s", path);
  char magic[8];
  long long np = 0, nc = 0;
  int valid = 0, job = RT_SUR_SIDE;
  float scal[S_LOSS], geo[4];
  rt_gate_opts gate;
  std::vector<float> h(NPARAM);
  std::vector<unsigned char> map(NCELLS);
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "RTMLP05", 8) == 0 && fread(&np, sizeof(np), 1, f) == 1 &&
            np == NPARAM && fread(scal, sizeof(float), S_LOSS, f) == (size_t)S_LOSS &&
            fread(h.data(), sizeof(float), NPARAM, f) == (size_t)NPARAM && fread(&nc, sizeof(nc), 1, f) == 1 &&
            nc == NCELLS && fread(&valid, sizeof(valid), 1, f) == 1 && fread(&gate, sizeof(gate), 1, f) == 1 &&
            fread(map.data(), 1, NCELLS, f) == (size_t)NCELLS && fread(&job, sizeof(int), 1, f) == 1 &&
            fread(geo, sizeof(float), 4, f) == 4 && (job == RT_SUR_SIDE || job == RT_SUR_CAP);
  fclose(f);
  if (!ok) return fail(RT_E_INVALID, "%s is not a surrogate file of this layout", path);
  rt_model mo = nullptr;
  int e = rt_surrogate_create(0, &mo);
  if (e) return e;
  e = rt_surrogate_set_scaling(mo, scal);
  if (!e) e = rt_surrogate_set_params(mo, h.data());
  if (!e) {
    mo->h_map = map;
    mo->map_valid = valid;
    mo->gate = gate;
    mo->job = job;
    memcpy(mo->geo, geo, sizeof(geo));
    e = upload_map(mo);
  }
  if (e) {
    rt_surrogate_free(mo);
    return e;
  }
  *out = mo;
  return RT_OK;
}

}  // extern "C"
