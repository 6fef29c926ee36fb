// Small-axis Gram matrix G = X^T X of a CSR cells x genes matrix (FP32 MFMA).
//
// The Gram of the gene axis (S_l = mat_l[D] mat_l[D]^T of the problem setup,
// formed only for the small axis; the large axis is reached through its
// singular vectors, Algorithm 1's first loop).  No centring or scaling.
//
// Two paths (picked from the shape, see gram_use_sparse): a sparse one that
// multiplies only each row's nonzeros (further below), and dense panels:
// row panels of X are densified into HBM (zero-padded to a multiple
// of 256 genes), then a symmetric rank-k update runs on the FP32 MFMA
// (32x32x2): one 256 x 256 output tile per workgroup of 16 waves (64 x 64
// each), only tiles with J >= I,
// 32-row chunks staged through LDS (double buffered).  Each workgroup folds
// its FP32 accumulators into an FP64 partial sum every 2048 rows, so the
// FP32 rounding error of a sum grows with at most 2048 terms; long K ranges
// are split across workgroups (one FP64 partial per split).  A final kernel
// adds the splits in fixed order, mirrors the upper triangle and rounds to
// FP32.  Results are deterministic for CSR input without duplicate columns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "gmgm_internal.h"
#include "mfma_util.h"

namespace gmgm_gr {

constexpr int GT = 256;           // output tile edge
constexpr int KC = 32;            // rows per LDS stage
constexpr int LST = 288;          // LDS row stride (floats): rows k and k+1 fall in disjoint bank halves
constexpr int FLUSH_CHUNKS = 64;  // FP32 -> FP64 fold period: 64 * 32 = 2048 rows
constexpr int THREADS = 1024;    // 16 waves, each a 64 x 64 block of the tile

struct TileArgs {
  const float* D;      // panel: rows_pad x pp, row-major, zero padded
  int64_t pp;          // padded gene count (multiple of GT)
  int64_t rows_pad;    // panel rows (multiple of KC)
  int64_t rows_split;  // rows per split (multiple of KC)
  const int2* tiles;   // (I, J), J >= I
  double* P;           // n_split x pp x pp FP64 partials
};

__global__ void __launch_bounds__(THREADS) gram_tile_kernel(TileArgs a) {
  __shared__ float lds[2][2][KC][LST];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 2, wc = w & 3, half = lane >> 5, l32 = lane & 31;
  const int2 IJ = a.tiles[blockIdx.x];
  const int s = blockIdx.y;
  const int64_t k_begin = (int64_t)s * a.rows_split;
  const int64_t k_end = k_begin + a.rows_split < a.rows_pad ? k_begin + a.rows_split : a.rows_pad;
  if (k_begin >= k_end) return;
  const int nchunks = (int)((k_end - k_begin) / KC);
  const float* Abase = a.D + (size_t)k_begin * a.pp + (size_t)IJ.x * GT;
  const float* Bbase = a.D + (size_t)k_begin * a.pp + (size_t)IJ.y * GT;

  // staging: thread t moves float4s q = t and q = t + 1024 of each 32 x 256 operand chunk
  const int q0 = tid, q1 = tid + THREADS;
  const size_t g0 = (size_t)(q0 >> 6) * a.pp + 4 * (q0 & 63), g1 = (size_t)(q1 >> 6) * a.pp + 4 * (q1 & 63);
  float4 ra0, ra1, rb0, rb1;
  auto load = [&](int c) {
    const size_t off = (size_t)c * KC * a.pp;
    ra0 = *reinterpret_cast<const float4*>(Abase + off + g0);
    ra1 = *reinterpret_cast<const float4*>(Abase + off + g1);
    rb0 = *reinterpret_cast<const float4*>(Bbase + off + g0);
    rb1 = *reinterpret_cast<const float4*>(Bbase + off + g1);
  };
  auto store = [&](int buf) {
    *reinterpret_cast<float4*>(&lds[buf][0][q0 >> 6][4 * (q0 & 63)]) = ra0;
    *reinterpret_cast<float4*>(&lds[buf][0][q1 >> 6][4 * (q1 & 63)]) = ra1;
    *reinterpret_cast<float4*>(&lds[buf][1][q0 >> 6][4 * (q0 & 63)]) = rb0;
    *reinterpret_cast<float4*>(&lds[buf][1][q1 >> 6][4 * (q1 & 63)]) = rb1;
  };

  v16f acc[2][2];
  auto zero_acc = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
  };
  double* Pt = a.P + (size_t)s * a.pp * a.pp + (size_t)IJ.x * GT * a.pp + (size_t)IJ.y * GT;
  auto fold = [&]() {
    // an opaque copy of the row stride keeps the 64 destination addresses from
    // being hoisted out of the K loop (they would not fit the register budget)
    int ld = (int)a.pp;
    asm volatile("" : "+s"(ld));
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wr * 64 + i * 32 + acc_row(v, half);
          const int col = wc * 64 + j * 32 + l32;
          double* dst = Pt + (size_t)row * ld + col;
          *dst = *dst + (double)acc[i][j][v];
          // keep at most four read-modify-writes in flight (register budget)
          if (v % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
  };

  zero_acc();
  load(0);
  store(0);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunks) load(c + 1);
#pragma unroll
    for (int kk = 0; kk < KC / 2; ++kk) {
      const int k = 2 * kk + half;
      float av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = lds[buf][0][k][wr * 64 + i * 32 + l32];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = lds[buf][1][k][wc * 64 + j * 32 + l32];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
      // operands of at most two K steps ahead: 4 MFMAs (256 cycles) hide an LDS read
      if (kk % 2 == 1) __builtin_amdgcn_sched_barrier(0);
    }
    if ((c + 1) % FLUSH_CHUNKS == 0 || c + 1 == nchunks) {
      fold();
      zero_acc();
    }
    if (c + 1 < nchunks) store(buf ^ 1);
    __syncthreads();
  }
}

// Zero-fill of n floats (n multiple of 4) / n doubles.
__global__ void fill_f32_kernel(float4* __restrict__ p, int64_t n4) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}
__global__ void fill_f64_kernel(double2* __restrict__ p, int64_t n2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

// Scatter CSR rows [r0, r0 + rows) into the zeroed panel (one wave per row).
// Malformed rows (row_ptr decreasing or beyond nnz, column outside [0, p)) are
// skipped and reported; duplicate columns add up.
__global__ void __launch_bounds__(256) densify_kernel(const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      const float* __restrict__ val, int64_t nnz,
                                                      int64_t p, int64_t r0, int64_t rows,
                                                      int64_t pp, float* __restrict__ D,
                                                      int* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= rows) return;
  const int64_t b = rp[r0 + i], e = rp[r0 + i + 1];
  if (b < 0 || e < b || e > nnz) {
    if (lane == 0) atomicCAS(status, 0, DEV_BADINDEX);
    return;
  }
  bool badc = false, badv = false;
  float* row = D + (size_t)i * pp;
  for (int64_t t = b + lane; t < e; t += 64) {
    const int c = col[t];
    const float v = val ? val[t] : 1.0f;
    if (c < 0 || c >= p) {
      badc = true;
      continue;
    }
    badv |= !isfinite(v);
    unsafeAtomicAdd(row + c, v);
  }
  if (__ballot(badc) && lane == 0) atomicCAS(status, 0, DEV_BADINDEX);
  if (__ballot(badv) && lane == 0) atomicCAS(status, 0, DEV_NONFINITE);
}

// G (p x p, row-major FP32) from the FP64 split partials: sum the splits in
// order, take the upper triangle's value for both (a, b) and (b, a).  With a
// shift z (the Gram of X + 1 z^T, cs = X's column sums): + cs_a z_b + z_a cs_b
// + n z_a z_b, in FP64 before rounding.
__global__ void __launch_bounds__(256) gram_finish_kernel(const double* __restrict__ P, int n_split,
                                                          int64_t pp, int64_t p,
                                                          const double* __restrict__ zs,
                                                          const double* __restrict__ cs, double nrows,
                                                          float* __restrict__ G) {
  __shared__ double t[32][33];
  const int A = blockIdx.y, B = blockIdx.x;
  const int lo = A < B ? A : B, hi = A < B ? B : A;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const size_t idx = (size_t)(lo * 32 + r) * pp + hi * 32 + tx;
    double s = 0.0;
    for (int q = 0; q < n_split; ++q) s += P[(size_t)q * pp * pp + idx];
    t[r][tx] = s;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t a = (int64_t)A * 32 + r, b = (int64_t)B * 32 + tx;
    if (a >= p || b >= p) continue;
    double v;
    if (A < B) v = t[r][tx];
    else if (A > B) v = t[tx][r];
    else v = r <= tx ? t[r][tx] : t[tx][r];
    if (zs) v += cs[a] * zs[b] + zs[a] * cs[b] + nrows * zs[a] * zs[b];
    G[a * p + b] = (float)v;
  }
}

// ------------------------------------------------------------------ sparse path
// G accumulated straight from the nonzeros: for every row x_r, the products
// x_ra x_rb of its entries with a <= b are added into 128 x 128 FP64 tiles
// held in LDS (one workgroup per tile pair (A, B), A <= B, and row split).
// Work is sum_r nnz_r^2 / 2 products instead of n p^2 / 2 for dense panels.
// The nonzeros are first copied block-major: the entries of column block q
// for all rows, row after row (a one-byte column within the block and the
// value), so that a tile pair reads two contiguous streams.  Finding each
// row's block boundaries needs strictly increasing columns per row; other
// rows (unsorted or duplicate columns) take every ordered pair with global
// FP64 atomics.
constexpr int ST = 128;               // sparse tile edge (FP64 tile: 128 KB of LDS)
constexpr int SP_THREADS = 1024;
constexpr int SCAN_T = 1024;          // rows per scan chunk

// One wave per row of [r0, r0 + rows): block offsets within the row,
// off[q][i] = number of the row's entries with column < q * ST (q = 0..nb),
// for sorted rows; zero offsets (no work) for every other row.  Unsorted rows
// are listed for the generic kernel, malformed rows reported and skipped.
__global__ void __launch_bounds__(256) block_offsets_kernel(const int64_t* __restrict__ rp,
                                                            const int32_t* __restrict__ col,
                                                            const float* __restrict__ val, int64_t nnz,
                                                            int64_t p, int64_t r0, int64_t rows, int nb,
                                                            int* __restrict__ off, int* __restrict__ bad_rows,
                                                            int* __restrict__ bad_count, int* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= rows) return;
  const int64_t b = rp[r0 + i], e = rp[r0 + i + 1];
  auto zero_offsets = [&]() {
    for (int q = lane; q <= nb; q += 64) off[(size_t)q * rows + i] = 0;
  };
  if (b < 0 || e < b || e > nnz || e - b > (int64_t)0x7fffffff) {
    if (lane == 0) atomicCAS(status, 0, DEV_BADINDEX);
    zero_offsets();
    return;
  }
  bool badc = false, badv = false, unsorted = false;
  for (int64_t t = b + lane; t < e; t += 64) {
    const int c = col[t];
    badc |= c < 0 || c >= p;
    if (val) badv |= !isfinite(val[t]);
    if (t > b) unsorted |= c <= col[t - 1];
  }
  if (__ballot(badv) && lane == 0) atomicCAS(status, 0, DEV_NONFINITE);
  if (__ballot(badc)) {
    if (lane == 0) atomicCAS(status, 0, DEV_BADINDEX);
    zero_offsets();
    return;
  }
  if (__ballot(unsorted)) {
    zero_offsets();
    if (lane == 0) bad_rows[atomicAdd(bad_count, 1)] = (int)(r0 + i);
    return;
  }
  // block q starts at the first entry whose column is >= q * ST
  for (int64_t t = b + lane; t < e; t += 64) {
    const int bc = col[t] / ST;
    const int bp = t > b ? col[t - 1] / ST : -1;
    for (int q = bp + 1; q <= bc; ++q) off[(size_t)q * rows + i] = (int)(t - b);
  }
  const int last = e > b ? col[e - 1] / ST : -1;
  for (int q = last + 1 + lane; q <= nb; q += 64) off[(size_t)q * rows + i] = (int)(e - b);
}

// Exclusive scan of SCAN_T values per workgroup (16 waves); returns the
// thread's exclusive prefix and leaves the workgroup total in *total.
__device__ inline unsigned block_exclusive_scan(unsigned v, unsigned* wsum, unsigned* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (threadIdx.x < 64) {
    const unsigned s = lane < 16 ? wsum[lane] : 0u;
    unsigned inc = s;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const unsigned y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane < 16) wsum[16 + lane] = inc - s;
    if (lane == 15) wsum[32] = inc;
  }
  __syncthreads();
  const unsigned r = x - v + wsum[16 + w];
  *total = wsum[32];
  __syncthreads();
  return r;
}

// Segment starts per (block q, row r) relative to the block's region, within
// a chunk of SCAN_T rows: S[q][r] (row stride rows + 1); chunk sums into
// tot[q][chunk].  Grid (chunks, nb).
__global__ void __launch_bounds__(SCAN_T) seg_scan_kernel(const int* __restrict__ off, int64_t rows,
                                                          int nchunks, unsigned* __restrict__ S,
                                                          unsigned* __restrict__ tot) {
  __shared__ unsigned wsum[33];
  const int q = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * SCAN_T + threadIdx.x;
  const unsigned c = r < rows ? (unsigned)(off[(size_t)(q + 1) * rows + r] - off[(size_t)q * rows + r]) : 0u;
  unsigned total;
  const unsigned ex = block_exclusive_scan(c, wsum, &total);
  if (r < rows) S[(size_t)q * (rows + 1) + r] = ex;
  if (threadIdx.x == 0) tot[(size_t)q * nchunks + blockIdx.x] = total;
}

// Per block q (one workgroup each): the chunk sums scanned in place into
// chunk bases; T[q] = the block's entry count.
__global__ void __launch_bounds__(SCAN_T) chunk_base_kernel(unsigned* __restrict__ tot, int nchunks,
                                                            unsigned long long* __restrict__ T) {
  __shared__ unsigned wsum[33];
  const int q = blockIdx.x;
  unsigned carry = 0;
  for (int c0 = 0; c0 < nchunks; c0 += SCAN_T) {
    const int c = c0 + (int)threadIdx.x;
    const unsigned v = c < nchunks ? tot[(size_t)q * nchunks + c] : 0u;
    unsigned total;
    const unsigned ex = block_exclusive_scan(v, wsum, &total);
    if (c < nchunks) tot[(size_t)q * nchunks + c] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) T[q] = carry;
}

// Region starts R0[q] = sum of T over blocks before q (one thread; nb <= 512),
// and the end sentinel S[q][rows] = T[q].
__global__ void region_kernel(const unsigned long long* __restrict__ T, int nb, int64_t rows,
                              unsigned long long* __restrict__ R0, unsigned* __restrict__ S) {
  if (threadIdx.x == 0) {
    unsigned long long acc = 0;
    for (int q = 0; q < nb; ++q) {
      R0[q] = acc;
      acc += T[q];
    }
  }
  for (int q = threadIdx.x; q < nb; q += blockDim.x) S[(size_t)q * (rows + 1) + rows] = (unsigned)T[q];
}

// S[q][r] += the base of r's chunk (absolute within the block's region).
__global__ void seg_add_kernel(unsigned* __restrict__ S, const unsigned* __restrict__ tot, int64_t rows, int nb,
                               int nchunks) {
  const int64_t total = (int64_t)nb * rows;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(x / rows);
    const int64_t r = x - (int64_t)q * rows;
    S[(size_t)q * (rows + 1) + r] += tot[(size_t)q * nchunks + r / SCAN_T];
  }
}

// The block-major copy: one wave per row; entry t of a sorted row goes to
// R0[q] + S[q][r] + (its rank within the row's block-q segment).  Rows whose
// segments are empty (unsorted, malformed) copy nothing.
__global__ void __launch_bounds__(256) block_scatter_kernel(const int64_t* __restrict__ rp,
                                                            const int32_t* __restrict__ col,
                                                            const float* __restrict__ val, int64_t nnz,
                                                            int64_t p, int64_t r0, int64_t rows,
                                                            const int* __restrict__ off,
                                                            const unsigned* __restrict__ S,
                                                            const unsigned long long* __restrict__ R0,
                                                            uint8_t* __restrict__ bcol, float* __restrict__ bval) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= rows) return;
  const int64_t b = rp[r0 + i], e = rp[r0 + i + 1];
  if (b < 0 || e < b || e > nnz) return;
  for (int64_t t = b + lane; t < e; t += 64) {
    const int c = col[t];
    if (c < 0 || c >= p) continue;
    const int q = c / ST;
    const unsigned s0 = S[(size_t)q * (rows + 1) + i], s1 = S[(size_t)q * (rows + 1) + i + 1];
    const int64_t rel = (t - b) - off[(size_t)q * rows + i];
    if (rel < 0 || rel >= (int64_t)(s1 - s0)) continue;
    const unsigned long long d = R0[q] + s0 + (unsigned long long)rel;
    bcol[d] = (uint8_t)(c - q * ST);
    bval[d] = val ? val[t] : 1.0f;
  }
}

struct SparseArgs {
  const unsigned* S;              // nb x (rows + 1) segment starts (relative to each block's region)
  const unsigned long long* R0;   // region start of each block
  const uint8_t* bcol;            // block-major copy: column within the block
  const float* bval;              //                   value
  int64_t rows;                   // rows of this chunk
  int64_t rows_split;             // rows per split
  const int2* tiles;              // (A, B), B >= A
  int64_t pp;                     // nb * ST
  double* P;                      // n_split x pp x pp FP64 partials (added to)
};

__global__ void __launch_bounds__(SP_THREADS) gram_sparse_tile_kernel(SparseArgs a) {
  __shared__ double t[ST * ST];
  const int tid = threadIdx.x;
  const int2 AB = a.tiles[blockIdx.x];
  const int A = AB.x, B = AB.y;
  const bool diag = A == B;
  for (int q = tid; q < ST * ST; q += SP_THREADS) t[q] = 0.0;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.y * a.rows_split;
  const int64_t hi = lo + a.rows_split < a.rows ? lo + a.rows_split : a.rows;
  const unsigned* SA = a.S + (size_t)A * (a.rows + 1);
  const unsigned* SB = a.S + (size_t)B * (a.rows + 1);
  const uint8_t* colA = a.bcol + a.R0[A];
  const float* valA = a.bval + a.R0[A];
  const uint8_t* colB = a.bcol + a.R0[B];
  const float* valB = a.bval + a.R0[B];
  for (int64_t r = lo + tid; r < hi; r += SP_THREADS) {
    const unsigned a0 = SA[r], a1 = SA[r + 1], b0 = SB[r], b1 = SB[r + 1];
    if (a0 >= a1 || b0 >= b1) continue;
    // eight B entries in registers at a time, every A entry against them
    for (unsigned j0 = b0; j0 < b1; j0 += 8) {
      int cb[8];
      double vb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const unsigned j = j0 + u < b1 ? j0 + u : b1 - 1;
        cb[u] = colB[j];
        vb[u] = (double)valB[j];
      }
      const unsigned iend = diag ? (a1 < j0 + 8 ? a1 : j0 + 8) : a1;   // diagonal tile: i <= j
      for (unsigned i = a0; i < iend; ++i) {
        const double va = (double)valA[i];
        double* trow = t + (int)colA[i] * ST;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const unsigned j = j0 + u;
          if (j < b1 && (!diag || j >= i)) atomicAdd(trow + cb[u], va * vb[u]);
        }
      }
    }
  }
  __syncthreads();
  double* Pt = a.P + (size_t)blockIdx.y * a.pp * a.pp + (size_t)A * ST * a.pp + (size_t)B * ST;
  for (int q = tid; q < ST * ST; q += SP_THREADS) {
    const int x = q / ST, y = q % ST;
    if (t[q] != 0.0) Pt[(size_t)x * a.pp + y] += t[q];
  }
}

// Rows without strictly increasing columns: every ordered pair (i, j) adds
// x_i x_j to P[c_i][c_j] when c_i <= c_j (so a duplicate column c gets
// (sum of its values)^2), with global FP64 atomics into partial 0.  One
// workgroup per listed row.
__global__ void __launch_bounds__(256) gram_rows_generic_kernel(const int64_t* __restrict__ rp,
                                                                const int32_t* __restrict__ col,
                                                                const float* __restrict__ val,
                                                                const int* __restrict__ list,
                                                                const int* __restrict__ count, int64_t pp,
                                                                double* __restrict__ P) {
  const int cnt = *count;
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) {
    const int64_t r = list[q];
    const int64_t b = rp[r], m = rp[r + 1] - b;
    for (int64_t x = threadIdx.x; x < m * m; x += blockDim.x) {
      const int64_t i = b + x / m, j = b + x % m;
      const int ci = col[i], cj = col[j];
      if (ci > cj) continue;
      const double v = (val ? (double)val[i] : 1.0) * (val ? (double)val[j] : 1.0);
      unsafeAtomicAdd(P + (size_t)ci * pp + cj, v);
    }
  }
}

inline unsigned grid_for(int64_t n, int per_block) {
  const int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

}  // namespace gmgm_gr

using namespace gmgm_gr;

// Path choice from the shape alone (no synchronisation): estimated time of
// the dense panels (FP32 MFMA, n p_pad^2 multiply-adds) against the sparse
// tiles (per tile pair a pass over the row offsets, the entries of both
// blocks re-read per pair, ~nnz^2 / 2n LDS atomics).  GMGM_GRAM_PATH=dense or
// =sparse in the environment forces a path.
static bool gram_use_sparse(int64_t n, int64_t p, int64_t nnz) {
  if (n >= ((int64_t)1 << 31)) return false;
  if (const char* e = getenv("GMGM_GRAM_PATH")) {
    if (!strcmp(e, "dense")) return false;
    if (!strcmp(e, "sparse")) return true;
  }
  const double nb = (double)((p + ST - 1) / ST);
  const double ppd = (double)((p + GT - 1) / GT * GT);
  const double t_dense = (double)n * ppd * ppd / 1.18e14;
  const double pairs = nb * (nb + 1) / 2;
  const double t_sparse = (pairs * (double)n * 24.0 + (nb + 1) * (double)nnz * 8.0) / 3.0e12 +
                          (double)nnz * (double)nnz / (2.0 * (double)n) / 1.0e13;
  return t_sparse < t_dense;
}

static gmgm_status gram_sparse(gmgm_ctx* c, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                               const int32_t* col, const float* val, const double* zs, const double* cs,
                               float* G) {
  hipStream_t st = c->stream;
  const int nb = (int)((p + ST - 1) / ST);
  const int64_t pp = (int64_t)nb * ST;
  const int n_pairs = nb * (nb + 1) / 2;
  // row chunks: offsets and segment starts of at most 2 GiB together
  const int64_t rows_c = std::min<int64_t>(n, std::max<int64_t>(SCAN_T, ((int64_t)1 << 31) / (8 * (nb + 1))));
  const int nchunks = (int)((rows_c + SCAN_T - 1) / SCAN_T);
  // row splits: enough workgroups to cover the chip, >= 4096 rows each, partials <= 8 GiB
  int n_split = (int)std::min<int64_t>(64, (2048 + n_pairs - 1) / n_pairs);
  n_split = (int)std::max<int64_t>(1, std::min<int64_t>(n_split, rows_c / 4096));
  while (n_split > 1 && (double)n_split * pp * pp * 8 > 8.0 * (1 << 30)) n_split--;

  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_off = up((size_t)(nb + 1) * rows_c * 4);
  const size_t b_S = up((size_t)nb * (rows_c + 1) * 4);
  const size_t b_tot = up((size_t)nb * nchunks * 4);
  const size_t b_T = up((size_t)nb * 8);
  const size_t b_bad = up((size_t)n * 4);
  void *wO, *wP, *wT, *wB;
  GMGM_TRY(ws_get(c, WS_GRAM0, 256 + b_off + b_S + b_tot + 2 * b_T + b_bad, &wO));
  GMGM_TRY(ws_get(c, WS_GRAM1, (size_t)n_split * pp * pp * sizeof(double), &wP));
  GMGM_TRY(ws_get(c, WS_GRAM2, (size_t)n_pairs * sizeof(int2), &wT));
  GMGM_TRY(ws_get(c, WS_GRAM3, up((size_t)std::max<int64_t>(nnz, 1) * 4) + up((size_t)std::max<int64_t>(nnz, 1)), &wB));
  char* w = (char*)wO;
  int* bad_count = (int*)w;
  int* off = (int*)(w + 256);
  unsigned* S = (unsigned*)(w + 256 + b_off);
  unsigned* tot = (unsigned*)(w + 256 + b_off + b_S);
  unsigned long long* T = (unsigned long long*)(w + 256 + b_off + b_S + b_tot);
  unsigned long long* R0 = (unsigned long long*)(w + 256 + b_off + b_S + b_tot + b_T);
  int* bad_rows = (int*)(w + 256 + b_off + b_S + b_tot + 2 * b_T);
  float* bval = (float*)wB;
  uint8_t* bcol = (uint8_t*)wB + up((size_t)std::max<int64_t>(nnz, 1) * 4);
  std::vector<int2> tiles;
  tiles.reserve(n_pairs);
  for (int A = 0; A < nb; ++A)
    for (int B = A; B < nb; ++B) tiles.push_back(make_int2(A, B));
  GMGM_HIP(c, hipMemcpyAsync(wT, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  GMGM_HIP(c, hipStreamSynchronize(st));   // the host vector must outlive the copy
  double* P = (double*)wP;
  const int64_t np2 = (int64_t)n_split * pp * pp / 2;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(np2, 256)), dim3(256), 0, st, (double2*)P, np2);
  hipLaunchKernelGGL(fill_f32_kernel, dim3(1), dim3(64), 0, st, (float4*)bad_count, (int64_t)1);
  for (int64_t r0 = 0; r0 < n; r0 += rows_c) {
    const int64_t rows = std::min<int64_t>(rows_c, n - r0);
    const int nch = (int)((rows + SCAN_T - 1) / SCAN_T);
    hipLaunchKernelGGL(block_offsets_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, row_ptr, col,
                       val, nnz, p, r0, rows, nb, off, bad_rows, bad_count, c->dev_status);
    hipLaunchKernelGGL(seg_scan_kernel, dim3((unsigned)nch, (unsigned)nb), dim3(SCAN_T), 0, st, off, rows, nch, S,
                       tot);
    hipLaunchKernelGGL(chunk_base_kernel, dim3((unsigned)nb), dim3(SCAN_T), 0, st, tot, nch, T);
    hipLaunchKernelGGL(region_kernel, dim3(1), dim3(256), 0, st, T, nb, rows, R0, S);
    hipLaunchKernelGGL(seg_add_kernel, dim3(grid_for((int64_t)nb * rows, 256)), dim3(256), 0, st, S, tot, rows, nb,
                       nch);
    hipLaunchKernelGGL(block_scatter_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, row_ptr, col, val,
                       nnz, p, r0, rows, off, S, R0, bcol, bval);
    SparseArgs sa{S, R0, bcol, bval, rows, (rows + n_split - 1) / n_split, (const int2*)wT, pp, P};
    hipEvent_t ev = timing_start(c);
    hipLaunchKernelGGL(gram_sparse_tile_kernel, dim3((unsigned)n_pairs, (unsigned)n_split), dim3(SP_THREADS), 0,
                       st, sa);
    timing_stop(c, ev);
  }
  hipLaunchKernelGGL(gram_rows_generic_kernel, dim3(256), dim3(256), 0, st, row_ptr, col, val, bad_rows,
                     bad_count, pp, P);
  const unsigned g32 = (unsigned)((p + 31) / 32);
  hipLaunchKernelGGL(gram_finish_kernel, dim3(g32, g32), dim3(256), 0, st, P, n_split, pp, p, zs, cs, (double)n, G);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

static gmgm_status gram_impl(gmgm_ctx* c, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                             const int32_t* col, const float* val, const double* zs, const double* cs, float* G) {
  if (n < 1 || p < 1 || p > 65536 || nnz < 0)
    return set_err(c, GMGM_E_SHAPE, "need n >= 1, 1 <= p <= 65536, nnz >= 0 (got n=%lld p=%lld nnz=%lld)",
                   (long long)n, (long long)p, (long long)nnz);
  if (!row_ptr || !G || (nnz > 0 && !col)) return set_err(c, GMGM_E_ARG, "null pointer argument");
  GMGM_HIP(c, hipSetDevice(c->device));
  if (gram_use_sparse(n, p, nnz)) return gram_sparse(c, n, p, nnz, row_ptr, col, val, zs, cs, G);
  hipStream_t st = c->stream;
  const int64_t pp = (p + GT - 1) / GT * GT;
  const int nt = (int)(pp / GT);
  const int n_tiles = nt * (nt + 1) / 2;
  // panel rows: about 2 GiB of densified rows per panel
  int64_t nb = ((int64_t)1 << 31) / (pp * 4) / KC * KC;
  nb = std::max<int64_t>(KC, std::min<int64_t>(nb, (n + KC - 1) / KC * KC));
  // K splits: enough workgroups to cover the chip, each split >= 256 rows,
  // partials at most 8 GiB
  int n_split = (int)std::min<int64_t>(64, (1024 + n_tiles - 1) / n_tiles);
  n_split = (int)std::max<int64_t>(1, std::min<int64_t>(n_split, nb / 256));
  while (n_split > 1 && (double)n_split * pp * pp * 8 > 8.0 * (1 << 30)) n_split--;

  void *wD, *wP, *wT;
  GMGM_TRY(ws_get(c, WS_GRAM0, (size_t)nb * pp * sizeof(float), &wD));
  GMGM_TRY(ws_get(c, WS_GRAM1, (size_t)n_split * pp * pp * sizeof(double), &wP));
  GMGM_TRY(ws_get(c, WS_GRAM2, (size_t)n_tiles * sizeof(int2), &wT));
  std::vector<int2> tiles;
  tiles.reserve(n_tiles);
  for (int I = 0; I < nt; ++I)
    for (int J = I; J < nt; ++J) tiles.push_back(make_int2(I, J));
  GMGM_HIP(c, hipMemcpyAsync(wT, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  // the host vector must outlive the copy
  GMGM_HIP(c, hipStreamSynchronize(st));
  float* D = (float*)wD;
  double* P = (double*)wP;
  const int64_t np2 = (int64_t)n_split * pp * pp / 2;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(np2, 256)), dim3(256), 0, st, (double2*)P, np2);
  for (int64_t r0 = 0; r0 < n; r0 += nb) {
    const int64_t rows = std::min<int64_t>(nb, n - r0);
    const int64_t rows_pad = (rows + KC - 1) / KC * KC;
    const int64_t n4 = rows_pad * pp / 4;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n4, 256)), dim3(256), 0, st, (float4*)D, n4);
    hipLaunchKernelGGL(densify_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, row_ptr, col, val,
                       nnz, p, r0, rows, pp, D, c->dev_status);
    const int64_t rs = ((rows_pad + n_split - 1) / n_split + KC - 1) / KC * KC;
    TileArgs ta{D, pp, rows_pad, rs, (const int2*)wT, P};
    hipEvent_t ev = timing_start(c);
    hipLaunchKernelGGL(gram_tile_kernel, dim3((unsigned)n_tiles, (unsigned)n_split), dim3(THREADS), 0, st, ta);
    timing_stop(c, ev);
  }
  const unsigned g32 = (unsigned)((p + 31) / 32);
  hipLaunchKernelGGL(gram_finish_kernel, dim3(g32, g32), dim3(256), 0, st, P, n_split, pp, p, zs, cs, (double)n, G);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_gram(gmgm_ctx_t c, int64_t n, int64_t p, int64_t nnz,
                                 const int64_t* row_ptr, const int32_t* col, const float* val,
                                 float* G) {
  GMGM_CHECK_CTX(c);
  return gram_impl(c, n, p, nnz, row_ptr, col, val, nullptr, nullptr, G);
}

extern "C" gmgm_status gmgm_gram_shifted(gmgm_ctx_t c, int64_t n, int64_t p, int64_t nnz,
                                         const int64_t* row_ptr, const int32_t* col, const float* val,
                                         const double* z, const double* csum, float* G) {
  GMGM_CHECK_CTX(c);
  if (!z || !csum) return set_err(c, GMGM_E_ARG, "null shift pointer");
  return gram_impl(c, n, p, nnz, row_ptr, col, val, z, csum, G);
}
