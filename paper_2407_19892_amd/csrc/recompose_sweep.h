// MFMA sweep of the fused recomposition + top-k (shared by the per-precision
// translation units that instantiate it).
//
// One workgroup = SW_WAVES waves; wave w keeps W (the psi-scaled rows of Psi it
// owns, TI tiles of 32 rows) in registers as the MFMA B operand for the whole
// sweep.  The 32-row tiles of V (the A operand, i.e. 32 columns of Psi) stream
// through double-buffered LDS, a few tiles per stage, loaded once per
// workgroup with coalesced 16-byte loads and read by every wave.  After each
// 32x32 MFMA tile a lane holds 16 values of one row of Psi (the accumulator
// column is the lane).  Each lane keeps a sorted top-C list (approximate
// |Psi_ij|, ascending j, ties to smaller j) of the row it owns and tests a
// whole tile against a threshold with one max and one compare.  The threshold
// is max(list's C-th value, list's k-th value - 2 beta_i), beta_i the row's
// rounding bound: a value below it can neither enter the list's top C nor come
// within 2 beta_i of the final k-th, so the final certificate (which takes the
// same maximum over the dropped values) still holds.
// Tiles where some lane has a value above it take the slow path: with two row
// tiles per wave the two accumulators' lane halves are exchanged so that every
// lane holds the 32 values of its own row, the values above the threshold are
// appended to the lane's own LDS queue (entry-major, lane-minor: no bank
// conflicts), and the queues are merged into the lists (all lanes at once)
// only when some lane's queue could overflow.
#pragma once

#include <hip/hip_runtime.h>

#include "gmgm_internal.h"
#include "mfma_util.h"

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace gmgm_rc {

constexpr int INVALID_J = 0x7fffffff;
constexpr int SW_WAVES = 8;                 // waves per workgroup (2 per SIMD)
constexpr int SW_THREADS = 64 * SW_WAVES;

struct SweepArgs {
  const u32x4* Vp;        // repacked V: n_vtiles tiles of UNITS*64 chunks
  const u32x4* Wp;        // repacked W: one tile per 32 local rows
  const int* ev;          // FP8: per V tile exponent
  const int* ew;          // FP8: per local W row exponent
  float* cval;            // candidates: [slot][split][sublist][C]
  int* cidx;
  const int* row_list;    // list mode: local row -> global row (nullptr: contiguous rows)
  const int* row_count;   // list mode: number of listed rows (device)
  int64_t n;
  int n_vtiles;
  int n_wtiles;           // contiguous mode: W tiles; list mode: capacity in tiles
  int64_t row0;           // contiguous mode: global row of local row 0
  int64_t row_begin, row_end;   // contiguous mode: rows whose lists are written
  int S, tiles_per_split;
  // per-row rounding bound beta_i = cprec ||W_i|| max_j ||V_j|| (rows from w_lo)
  const double* wnorm;
  const unsigned* vmax_bits;
  int64_t w_lo;
  double cprec;
  int k;
  // threshold mode: keep |Psi_ij| >= thr; cval / cidx hold capt candidates per
  // (slot, split, sub-list), tcount their counts (beyond capt: overflowed)
  double thr;
  int capt;
  int* tcount;
  const long long* toff;  // threshold mode, listed rows: candidate offsets per slot (null: slot * capt)
  // column tiles visited: jt0, jt0 + jt_stride, ... (0 or 1: every tile)
  int jt_stride;
  // symmetric form: tau[j] (n_vtiles * 32 entries) is a lower bound of row
  // j's final cut lowered by its rounding margin (+inf: none; padding +inf);
  // the row's own list starts from it, and values Psi_ij of the column side
  // above tau[j] go to a shared pool as (j, i, |Psi_ij|): a wave takes
  // cs_chunk entries at a time, at the start of a stage whose chunk has less
  // than half of them free (cs_next counts the entries handed out, up to
  // cs_cap), and records how many of a chunk it filled in cs_fill[chunk]
  const float* tau;
  int* cs_j;
  int* cs_i;
  float* cs_v;
  unsigned* cs_next;
  int cs_cap;             // below 2^31 - cs_chunk
  int cs_chunk;
  int* cs_fill;
  int* cs_overflow;       // set to 1 when entries were lost (the pool ran out, or a
                          // stage outgrew the half chunk its wave started with)
};


// HALF: split BF16 form only, the unit offset of the low parts (kpad / 16).
template <int PREC, int HALF = 0>
__device__ inline v16f mfma_chunk(const u32x4* a, const u32x4* b, v16f acc, int u) {
  if constexpr (PREC == P_BF16X3) {
    if (u < HALF) {
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a[u]),
                                                   __builtin_bit_cast(v8bf, b[u]), acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a[u]),
                                                   __builtin_bit_cast(v8bf, b[u + HALF]), acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a[u + HALF]),
                                                   __builtin_bit_cast(v8bf, b[u]), acc, 0, 0, 0);
    }
  } else if constexpr (PREC == P_F32) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[u][q]), __uint_as_float(b[u][q]),
                                                acc, 0, 0, 0);
  } else if constexpr (PREC == P_BF16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a[u]),
                                                 __builtin_bit_cast(v8bf, b[u]), acc, 0, 0, 0);
  } else {
    if ((u & 1) == 0) {
      v8i av = __builtin_bit_cast(v8i, __builtin_shufflevector(a[u], a[u + 1], 0, 1, 2, 3, 4, 5, 6, 7));
      v8i bv = __builtin_bit_cast(v8i, __builtin_shufflevector(b[u], b[u + 1], 0, 1, 2, 3, 4, 5, 6, 7));
      // format 0 = FP8 e4m3 for both operands, unit block scales (E8M0 127 = 2^0)
      acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc, 0, 0, 0, 127, 0, 127);
    }
  }
  return acc;
}

// Insert (v, j) into the descending list (lv, li) of length C; requires v > lv[C-1].
// Equal values keep their order, so with ascending j per lane ties go to smaller j.
// One downward pass: entry s takes entry s-1 when v beats entry s-1, v when v
// beats entry s only, else stays; only two comparison masks are live at a time.
template <int C>
__device__ inline void list_insert(float (&lv)[C], int (&li)[C], float v, int j) {
  bool g_hi = v > lv[C - 1];
#pragma unroll
  for (int s = C - 1; s > 0; --s) {
    const bool g_lo = v > lv[s - 1];       // entry s-1 is not yet updated
    const float nv = g_lo ? lv[s - 1] : (g_hi ? v : lv[s]);
    const int nj = g_lo ? li[s - 1] : (g_hi ? j : li[s]);
    lv[s] = nv;
    li[s] = nj;
    g_hi = g_lo;
  }
  lv[0] = g_hi ? v : lv[0];
  li[0] = g_hi ? j : li[0];
}

// Lane halves: after a 32x32 MFMA, lanes l and l + 32 hold the two halves
// (16 columns each) of the same row.  v_permlane32_swap exchanges the upper
// half of one register with the lower half of another; it is used to share
// per-lane scalars between the two halves.
__device__ inline void swap_halves(float& x, float& y) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}
__device__ inline void swap_halves(int& x, int& y) {
  auto r = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
  x = (int)r[0];
  y = (int)r[1];
}

// With two row tiles per wave ("pair" mode) lane l < 32 owns the list of row
// l of tile 0 and lane l + 32 the list of row l of tile 1 (whole rows); with
// one row tile each lane owns the list of its half row.
__host__ __device__ constexpr bool sweep_pairs(int TI) { return TI == 2; }
__host__ __device__ constexpr int sweep_nsub(int TI) { return sweep_pairs(TI) ? 1 : 2; }
// V tiles per LDS stage: at most 44 KB per stage buffer (fewer barriers).
__host__ __device__ constexpr int sweep_tps(int UNITS) { return 44 / UNITS > 0 ? 44 / UNITS : 1; }
constexpr int SW_Q = 16;  // append-queue entries per lane (own list), in LDS
static_assert(SW_Q >= 16, "the slow path appends up to 16 values per half row after a flush");

// The largest float below f (f finite or infinite).
__device__ inline float float_below(float f) {
  if (f == -INFINITY) return f;
  if (f == 0.0f) return -__int_as_float(1);
  const int b = __float_as_int(f);
  return __int_as_float(f > 0.0f ? b - 1 : b + 1);
}

struct QEntry {
  float v;
  int j;
};

// THR selects the threshold mode: the per-row threshold is fixed (the
// requested one lowered by the row's rounding bound) and every value above it
// is written straight to the row's candidate region; no lists are kept.
// SYM selects the symmetric form (Psi = Psi^T): workgroup b (rows of tiles
// [16b, 16b + 16)) visits only column tiles >= 16b, from the last one down
// (so the workgroups running together stream the same tiles, as in the full
// sweep, and share them in L2).  Inside its own block
// both orientations are visited by its own waves; beyond it, each computed
// value also serves row j of the column: it is kept for row j when it exceeds
// tau[j], a bound under which no value of row j can matter (so the row side
// of row j, which never visits columns of earlier blocks, misses nothing).
// STRIDED visits every a.jt_stride-th column tile only (a sample of the columns).
template <int PREC, int UNITS, int TI, int C, bool THR = false, bool SYM = false, bool STRIDED = false>
__global__ void __launch_bounds__(SW_THREADS) sweep_kernel(SweepArgs a) {
  static_assert(TI == 1 || TI == 2, "one or two row tiles per wave");
  static_assert(!THR || TI == 2, "threshold mode keeps whole rows per lane");
  static_assert(!SYM || (TI == 2 && !THR), "the symmetric form keeps whole rows per lane");
  constexpr bool PAIR = sweep_pairs(TI);
  constexpr int NSUB = sweep_nsub(TI);
  constexpr int TPS = sweep_tps(UNITS);
  constexpr int TILE_U = UNITS * 64;              // chunks per V tile
  constexpr int STAGE_U = TPS * TILE_U;           // chunks per stage
  constexpr int PF = (STAGE_U + SW_THREADS - 1) / SW_THREADS;
  constexpr int TAU_N = SYM ? TPS * 32 : 4;       // column bounds of a stage's tiles
  // two stage buffers as distinct objects: LDS reads of one are then known not
  // to alias the global-to-LDS loads in flight into the other
  __shared__ u32x4 lds_a[STAGE_U];
  __shared__ u32x4 lds_b[STAGE_U];
  __shared__ __attribute__((aligned(16))) float tau_a[TAU_N];
  __shared__ __attribute__((aligned(16))) float tau_b[TAU_N];
  // queue[wave][entry][lane]: each lane appends to its own column
  __shared__ QEntry queue[SW_WAVES][SW_Q][64];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the wave index is uniform within a wave: keep it (and all it derives) scalar
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int h = lane >> 5;
  const int l32 = lane & 31;
  const bool listed = a.row_list != nullptr;
  const int nrows_list = listed ? *a.row_count : 0;
  const int n_wt = listed ? (nrows_list + 31) / 32 : a.n_wtiles;
  const int wg_t0 = blockIdx.x * SW_WAVES * TI;
  if (wg_t0 >= n_wt) return;                      // whole workgroup idle (uniform)
  const int wt0 = wg_t0 + wave * TI;
  const bool active = wt0 < n_wt;                 // wave-uniform; idle waves still stage V

  u32x4 b[TI][UNITS];
  // 32-bit indices throughout (the host guarantees n < 2^31 - 64)
  const int n32 = (int)a.n;
  int myrow[TI];                                  // global row of this lane's values (-1: none)
  int slot[TI];                                   // candidate slot (-1: not written)
  int ewt[TI];
#pragma unroll
  for (int t = 0; t < TI; ++t) {
    const int wt = wt0 + t;
    const int64_t w = (int64_t)wt * 32 + l32;
    ewt[t] = 0;
    myrow[t] = -1;
    slot[t] = -1;
    if (wt < n_wt) {
#pragma unroll
      for (int u = 0; u < UNITS; ++u) b[t][u] = a.Wp[((int64_t)wt * UNITS + u) * 64 + lane];
      if constexpr (PREC == P_FP8) ewt[t] = a.ew[w];
      if (listed) {
        if (w < nrows_list) {
          myrow[t] = a.row_list[w];
          slot[t] = (int)w;
        }
      } else {
        myrow[t] = (int)(a.row0 + w);
        if (myrow[t] >= a.row_begin && myrow[t] < a.row_end) slot[t] = (int)(myrow[t] - a.row_begin);
      }
    } else {
#pragma unroll
      for (int u = 0; u < UNITS; ++u) b[t][u] = u32x4{0, 0, 0, 0};
    }
  }
  // contiguous mode: the wave's rows are tiles tile0 .. tile0 + TI - 1 of V
  const int tile0 = (int)(a.row0 >> 5) + wt0;

  // the list this lane owns, and the lists its values go to
  float lv[C];
  int li[C];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    lv[s] = -1.0f;
    li[s] = INVALID_J;
  }
  float tau[TI];       // threshold of the list of the row whose values this lane holds in tile t
#pragma unroll
  for (int t = 0; t < TI; ++t) tau[t] = -1.0f;
  int cnt = 0;         // entries in this lane's queue
  // the row of this lane's own list: row l32 of tile h (pairs) or of the lane's tile
  const int myrow_own = PAIR ? myrow[h == 0 ? 0 : TI - 1] : myrow[0];
  const int ew_own = PAIR ? ewt[h == 0 ? 0 : TI - 1] : ewt[0];
  // 2 beta of the own row (0 for lanes without a row)
  const double beta_own = myrow_own >= 0
      ? a.cprec * a.wnorm[myrow_own - a.w_lo] * (double)__uint_as_float(*a.vmax_bits)
      : 0.0;
  const float beta2 = (float)(2.0 * beta_own);
  float own_tau = -1.0f;   // max(lv[C-1], lv[k-1] - beta2), refreshed by flush
  // symmetric form: the own row's list starts from its bound (none: -1)
  float seed_own = -1.0f;
  if constexpr (SYM) {
    if (myrow_own >= 0 && myrow_own < n32) {
      const float t = a.tau[myrow_own];
      seed_own = t < INFINITY ? t : -1.0f;
    }
    own_tau = seed_own;
    float x = own_tau, y = own_tau;
    swap_halves(x, y);
    tau[0] = x;
    tau[TI - 1] = y;
  }
  // symmetric form: the wave's current pool chunk (-1: none yet, -2: the pool
  // ran out) and the entries it holds
  int cbase = -1;
  int cused = 0;
  // the candidate region this lane writes in threshold mode
  const int to = PAIR ? h : 0;
  const int sub = PAIR ? 0 : h;
  int64_t tbase = 0;
  int tcap = 0;         // candidate room of the own row (threshold mode)
  if constexpr (THR) {
    if (slot[to] >= 0) {
      tbase = a.toff ? a.toff[slot[to]] : (((int64_t)slot[to] * a.S + blockIdx.y) * NSUB + sub) * a.capt;
      tcap = a.toff ? (int)(a.toff[slot[to] + 1] - a.toff[slot[to]]) : a.capt;
    }
  }
  int tcnt = 0;
  if constexpr (THR) {
    // candidates: approximate |Psi| >= thr - beta (every exact |Psi| >= thr is
    // one); as a float compared with '>': the value just below thr - beta
    // rounded down.  Lanes without a written row take nothing.
    own_tau = INFINITY;
    if (slot[to] >= 0) {
      const double lo = a.thr - beta_own;
      float f = (float)lo;
      if ((double)f > lo) f = float_below(f);
      own_tau = float_below(f);
    }
    if constexpr (PAIR) {
      float x = own_tau, y = own_tau;
      swap_halves(x, y);
      tau[0] = x;
      tau[TI - 1] = y;
    } else {
      tau[0] = own_tau;
    }
  }

  // Merge every lane's queue into its list (all lanes at once), then refresh the
  // cached thresholds.  Wave-uniform.  A lane reads only the entries it wrote,
  // and a wave's LDS operations complete in order.
  auto flush = [&]() {
    int maxc = cnt;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxc = max(maxc, __shfl_xor(maxc, off, 64));
    for (int q = 0; q < maxc; ++q) {
      if (q < cnt) {
        const QEntry e = queue[wave][q][lane];
        if (e.v > lv[C - 1]) list_insert<C>(lv, li, e.v, e.j);
      }
    }
    cnt = 0;
    // the k-th entry of the descending list: the smallest of its first k entries
    // (compare and select; an index would move the list out of registers)
    float kth = lv[0];
#pragma unroll
    for (int q = 1; q < C; ++q) kth = (q < a.k && lv[q] < kth) ? lv[q] : kth;
    own_tau = fmaxf(lv[C - 1], kth - beta2);
    if constexpr (SYM) own_tau = fmaxf(own_tau, seed_own);
    if constexpr (PAIR) {
      float x = own_tau, y = own_tau;
      swap_halves(x, y);         // x: list of row l32 of tile 0, y: of tile 1
      tau[0] = x;
      tau[TI - 1] = y;
    } else {
      tau[0] = own_tau;
    }
  };

  // column tiles: [jt0, jt1) every jstride-th (symmetric form: from the
  // workgroup's first row tile on)
  const int jstride = STRIDED && a.jt_stride > 1 ? a.jt_stride : 1;
  const int jt0 = SYM ? (int)(a.row0 >> 5) + wg_t0 : blockIdx.y * a.tiles_per_split;
  const int jt1 = SYM ? a.n_vtiles : min(a.n_vtiles, jt0 + a.tiles_per_split);
  const int nl = jt1 > jt0 ? (jt1 - jt0 + jstride - 1) / jstride : 0;
  const int nst = (nl + TPS - 1) / TPS;
  // symmetric form: tiles from here on lie beyond the workgroup's own rows
  const int own_end = (int)(a.row0 >> 5) + wg_t0 + SW_WAVES * TI;

  // Stage loads go straight from global memory into LDS (global_load_lds,
  // 16 bytes per lane): lane l of a wave writes slot (its wave's base) + l, so
  // chunk idx lands at lds[buf][idx].  Chunks past the column range are not
  // loaded (their slots are never read).  The symmetric form also stages the
  // column bounds of the tiles (lanes 0 .. 8 TPS - 1 of wave 0, 16 bytes each).
  auto load_stage = [&](int st, u32x4* dst, float* tdst) {
    if constexpr (STRIDED) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int idx = tid + q * SW_THREADS;
        const int tl = idx / TILE_U;
        const int jl = st * TPS + tl;
        if (idx < STAGE_U && jl < nl) {
          const int64_t g = (int64_t)(jt0 + jl * jstride) * TILE_U + (idx - tl * TILE_U);
          __builtin_amdgcn_global_load_lds((const void*)(a.Vp + g),
                                           (__attribute__((address_space(3))) void*)(dst + (idx & ~63)), 16, 0, 0);
        }
      }
    } else {
      int64_t base, lim;
      if constexpr (SYM) {   // stages from the last column tile down
        const int hi = jt1 - st * TPS;
        base = (int64_t)max(jt0, hi - TPS) * TILE_U;
        lim = (int64_t)hi * TILE_U;
      } else {
        base = (int64_t)(jt0 + st * TPS) * TILE_U;
        lim = (int64_t)jt1 * TILE_U;
      }
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int idx = tid + q * SW_THREADS;
        const int64_t g = base + idx;
        if (idx < STAGE_U && g < lim)
          __builtin_amdgcn_global_load_lds((const void*)(a.Vp + g),
                                           (__attribute__((address_space(3))) void*)(dst + (idx & ~63)), 16, 0, 0);
      }
    }
    if constexpr (SYM) {
      // threads 0 .. 8 TPS - 1: the bounds, 16 bytes each (thread q lands at
      // float 4q: its wave's base plus 16 bytes per lane)
      static_assert(TPS * 8 <= SW_THREADS, "bound staging exceeds the workgroup");
      if (tid < TPS * 8) {
        const int hi = jt1 - st * TPS;
        const int jt = max(jt0, hi - TPS) + (tid >> 3);
        if (jt < hi)
          __builtin_amdgcn_global_load_lds((const void*)(a.tau + (int64_t)jt * 32 + 4 * (tid & 7)),
                                           (__attribute__((address_space(3))) void*)(tdst + 4 * (tid & ~63)), 16, 0,
                                           0);
      }
    }
  };

  // the MFMA sweep of stage st, whose V tiles are in rd (column bounds in trd)
  auto sweep_stage = [&](int st, const u32x4* rd, const float* trd) {
    if constexpr (SYM) {
      // a stage starts with at least half a chunk free in the wave's chunk
      // (taking chunks here keeps the pool's returning atomic out of the tile
      // loop, whose loads would otherwise wait for it)
      if (active && cbase != -2 && (cbase == -1 || 2 * cused > a.cs_chunk)) {
        if (cbase >= 0 && lane == 0) a.cs_fill[cbase / a.cs_chunk] = cused;
        unsigned got = 0;
        if (lane == 0) got = atomicAdd(a.cs_next, (unsigned)a.cs_chunk);
        got = (unsigned)__builtin_amdgcn_readfirstlane((int)got);
        if ((long long)got + a.cs_chunk > (long long)a.cs_cap) {
          if (lane == 0) atomicOr(a.cs_overflow, 1);
          cbase = -2;
        } else {
          cbase = (int)got;
        }
        cused = 0;
      }
    }
    if (active) {
#pragma unroll 1
      for (int tt = 0; tt < TPS; ++tt) {
        int jt;
        if constexpr (SYM) {
          const int hi = jt1 - st * TPS;
          jt = max(jt0, hi - TPS) + tt;
          if (jt >= hi) break;
        } else {
          const int jl = st * TPS + tt;
          if (jl >= nl) break;
          jt = jt0 + jl * jstride;
        }
        u32x4 av[UNITS];
#pragma unroll
        for (int u = 0; u < UNITS; ++u) av[u] = rd[tt * TILE_U + u * 64 + lane];
        v16f acc[TI];
#pragma unroll
        for (int t = 0; t < TI; ++t)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[t][v] = 0.0f;
#pragma unroll
        for (int u = 0; u < UNITS; ++u)
#pragma unroll
          for (int t = 0; t < TI; ++t) acc[t] = mfma_chunk<PREC, UNITS / 2>(av, b[t], acc[t], u);
        // issue every operand read of the tile before its MFMAs (else the
        // scheduler reuses one register and waits on each read in turn)
        constexpr int MF = PREC == P_F32 ? 4 * UNITS : PREC == P_FP8 ? UNITS / 2
                         : PREC == P_BF16X3 ? 3 * (UNITS / 2) : UNITS;
        __builtin_amdgcn_sched_group_barrier(0x100, UNITS, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, MF * TI, 0);

        const int j0 = jt * 32;
        // tiles holding the diagonal or the end of the columns exclude some values
        bool masked = j0 + 32 > n32;               // wave-uniform
        if (listed) {
          bool diag = false;
#pragma unroll
          for (int t = 0; t < TI; ++t) diag |= myrow[t] >= 0 && (myrow[t] >> 5) == jt;
          masked = masked || __ballot(diag) != 0;
        } else {
          masked = masked || (jt >= tile0 && jt < tile0 + TI);
        }
        // wave-uniform by construction; say so, so that it stays a scalar branch
        masked = __builtin_amdgcn_readfirstlane(masked ? 1 : 0) != 0;
        const int lim = n32 - j0;                  // columns at offsets >= lim do not exist
        int evt = 0;
        if constexpr (PREC == P_FP8) evt = a.ev[jt];

        // fast path: one max per (row tile) and one compare with the cached threshold
        float thr[TI], m[TI];
        bool pass[TI], any = false;
#pragma unroll
        for (int t = 0; t < TI; ++t) {
          float mm;
          if (masked) {
            const int d = myrow[t] - j0;           // the diagonal's offset in this tile
            mm = -1.0f;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int o = acc_row(v, h);
              mm = fmaxf(mm, (o < lim && o != d) ? fabsf(acc[t][v]) : -1.0f);
            }
          } else {
            mm = fabsf(acc[t][0]);
#pragma unroll
            for (int v = 1; v < 16; ++v) mm = fmaxf(mm, fabsf(acc[t][v]));
          }
          m[t] = mm;
          thr[t] = tau[t];
          if constexpr (PREC == P_FP8) thr[t] = __builtin_ldexpf(thr[t], -(ewt[t] + evt));
          pass[t] = mm > thr[t];
          any |= pass[t];
        }
        if constexpr (SYM) {
          // column side (tiles beyond the workgroup's own rows, never masked):
          // register v of this lane holds column j0 + acc_row(v, h) for the
          // wave's rows l32 (tile 0) and 32 + l32 (tile 1); group g of half h
          // is the four consecutive columns 8g + 4h .. 8g + 4h + 3
          if (jt >= own_end) {
            const float* tl = trd + tt * 32 + 4 * h;
            bool cg[4];   // some value of group g (columns 8g + 4h ..) beats its column's bound
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              const float4 tg = *(const float4*)(tl + 8 * g);
              cg[g] = fmaxf(fabsf(acc[0][4 * g]), fabsf(acc[TI - 1][4 * g])) > tg.x;
              cg[g] |= fmaxf(fabsf(acc[0][4 * g + 1]), fabsf(acc[TI - 1][4 * g + 1])) > tg.y;
              cg[g] |= fmaxf(fabsf(acc[0][4 * g + 2]), fabsf(acc[TI - 1][4 * g + 2])) > tg.z;
              cg[g] |= fmaxf(fabsf(acc[0][4 * g + 3]), fabsf(acc[TI - 1][4 * g + 3])) > tg.w;
            }
            if (__ballot(cg[0] || cg[1] || cg[2] || cg[3])) {
#pragma unroll
              for (int g = 0; g < 4; ++g) {
                if (!__ballot(cg[g])) continue;
                const float4 tg = *(const float4*)(tl + 8 * g);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const int v = 4 * g + e;
                  const float te = e == 0 ? tg.x : e == 1 ? tg.y : e == 2 ? tg.z : tg.w;
#pragma unroll
                  for (int t = 0; t < TI; ++t) {
                    const float x = fabsf(acc[t][v]);
                    const bool take = x > te && myrow[t] >= 0 && myrow[t] < n32;
                    const unsigned long long mk = __ballot(take);
                    if (mk) {
                      const int m = (int)__popcll(mk);
                      if (cbase >= 0 && cused + m > a.cs_chunk) {
                        // more than the room the stage started with: the
                        // call falls back to the full sweep
                        if (lane == 0) atomicOr(a.cs_overflow, 1);
                        cbase = -2;
                      }
                      if (cbase >= 0) {
                        const int pos = cbase + cused + (int)__builtin_amdgcn_mbcnt_hi(
                                                (unsigned)(mk >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
                        if (take) {
                          a.cs_j[pos] = j0 + acc_row(v, h);
                          a.cs_i[pos] = myrow[t];
                          a.cs_v[pos] = x;
                        }
                        cused += m;
                      }
                    }
                  }
                }
              }
            }
          }
        }
        if (__ballot(any)) {
          // own-row values: with two row tiles, exchange the accumulators' lane
          // halves so that acc[0] / acc[1] hold columns acc_row(v, 0) / acc_row(v, 1)
          // of this lane's own row; with one tile, acc[0] holds half h of it
          // the row maxima go through the same exchange: mh[c] is then the
          // largest value of half c of the own row, and a half that no lane
          // needs is skipped
          float mh0 = m[0], mh1 = m[TI - 1];
          if constexpr (PAIR) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              float p0 = acc[0][v], p1 = acc[TI - 1][v];
              swap_halves(p0, p1);
              acc[0][v] = p0;
              acc[TI - 1][v] = p1;
            }
            swap_halves(mh0, mh1);
          }
          int sc = 0;   // FP8: the scale exponent of this lane's own values
          if constexpr (PREC == P_FP8) sc = ew_own + evt;
          float own = own_tau;
          if constexpr (PREC == P_FP8) own = __builtin_ldexpf(own, -sc);
          if constexpr (THR) {
            // threshold mode: both halves of the own row, emitted in ascending
            // column order (group g of half 0 holds columns 8g..8g+3, of half
            // 1 columns 8g+4..8g+7)
            float x[2][16];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
#pragma unroll
              for (int v = 0; v < 16; ++v) {
                const float y = fabsf(hh ? acc[TI - 1][v] : acc[0][v]);
                const int o = acc_row(v, hh);
                x[hh][v] = (masked && (o >= lim || o == myrow_own - j0)) ? -INFINITY : y;
              }
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
              for (int hh = 0; hh < 2; ++hh) {
                const float gmx = fmaxf(fmaxf(x[hh][4 * g], x[hh][4 * g + 1]), fmaxf(x[hh][4 * g + 2], x[hh][4 * g + 3]));
                if (!__ballot(gmx > own)) continue;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const int v = 4 * g + e;
                  float xv = x[hh][v];
                  const bool take = xv > own;
                  if constexpr (PREC == P_FP8) xv = __builtin_ldexpf(xv, sc);
                  if (take && tcnt < tcap) {
                    a.cval[tbase + tcnt] = xv;
                    a.cidx[tbase + tcnt] = j0 + acc_row(v, hh);
                  }
                  tcnt += take ? 1 : 0;
                }
              }
          } else
#pragma unroll
          for (int hh = 0; hh < (PAIR ? 2 : 1); ++hh) {
            if (PAIR && !__ballot((hh ? mh1 : mh0) > own)) continue;
            const int colh = PAIR ? hh : h;
            float x[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) x[v] = fabsf((PAIR && hh) ? acc[TI - 1][v] : acc[0][v]);
            if (masked) {
              const int d = myrow_own - j0;
#pragma unroll
              for (int v = 0; v < 16; ++v) {
                const int o = acc_row(v, colh);
                x[v] = (o >= lim || o == d) ? -INFINITY : x[v];   // below every threshold
              }
            }
            float gm[4];
            int need = 0;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              gm[g] = fmaxf(fmaxf(x[4 * g], x[4 * g + 1]), fmaxf(x[4 * g + 2], x[4 * g + 3]));
              need += gm[g] > own ? 4 : 0;
            }
            // every lane writes at index cnt + (its takes so far) in each group the
            // wave enters: with cnt + need <= SW_Q - 1, or an empty queue and
            // need <= 16 = SW_Q, no write leaves the lane's SW_Q entries
            if (__ballot(cnt > 0 && cnt + need >= SW_Q)) {
              flush();
              own = own_tau;
              if constexpr (PREC == P_FP8) own = __builtin_ldexpf(own, -sc);
            }
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              if (!__ballot(gm[g] > own)) continue;
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int v = 4 * g + e;
                float xv = x[v];
                const bool take = xv > own;
                if constexpr (PREC == P_FP8) xv = __builtin_ldexpf(xv, sc);
                // written unconditionally, kept only if taken
                queue[wave][cnt][lane] = QEntry{xv, j0 + acc_row(v, colh)};
                cnt += take ? 1 : 0;
              }
            }
          }
        }
      }
    }
  };

  if (nst > 0) load_stage(0, lds_a, tau_a);
  // every prologue load (the B operands, stage 0) has landed
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // stages alternate between the buffers; the other buffer was last read in the
  // previous stage, which every wave has left at the barrier
  for (int st = 0; st < nst; st += 2) {
    if (st + 1 < nst) load_stage(st + 1, lds_b, tau_b);  // lands in LDS during the MFMAs
    sweep_stage(st, lds_a, tau_a);
    __builtin_amdgcn_s_waitcnt(0);                // this wave's loads have landed
    __syncthreads();                              // and everyone's
    if (st + 1 >= nst) break;
    if (st + 2 < nst) load_stage(st + 2, lds_a, tau_a);
    sweep_stage(st + 1, lds_b, tau_b);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  if constexpr (SYM) {
    if (cbase >= 0 && lane == 0) a.cs_fill[cbase / a.cs_chunk] = cused;
  }
  if (!active) return;
  if constexpr (THR) {
    if (slot[to] >= 0) a.tcount[((int64_t)slot[to] * a.S + blockIdx.y) * NSUB + sub] = tcnt;
    return;
  }
  flush();
  // the list of this lane: row l32 of tile h (pairs) or this lane's half row
  if (slot[to] >= 0) {
    const int64_t base = (((int64_t)slot[to] * a.S + blockIdx.y) * NSUB + sub) * C;
#pragma unroll
    for (int s = 0; s < C; ++s) {
      a.cval[base + s] = lv[s];
      a.cidx[base + s] = li[s];
    }
  }
}

typedef void (*SweepFn)(SweepArgs);

// Row tiles per wave: two for the short BF16 / FP8 operands (each lane then
// owns one full row), one for FP32 and split BF16 operands (lanes keep half
// rows); this is the register budget of the B operands and lists at 2 waves
// per SIMD.
__host__ __device__ constexpr int ti_for(int prec, int C) {
  return (prec == P_BF16 || prec == P_FP8) ? 2 : 1;
}

// One translation unit per (precision, list length) keeps the build parallel.
SweepFn pick_sweep_f32_c16(int kpad);
SweepFn pick_sweep_f32_c32(int kpad);
SweepFn pick_sweep_bf16_c16(int kpad);
SweepFn pick_sweep_bf16_c32(int kpad);
SweepFn pick_sweep_fp8_c16(int kpad);
SweepFn pick_sweep_fp8_c32(int kpad);
SweepFn pick_sweep_bf16x3(int kpad, int C);   // split BF16 re-sweep
SweepFn pick_sweep_thr(int prec, int kpad);   // threshold mode
SweepFn pick_sweep_bf16_sym(int kpad, int C); // symmetric form
SweepFn pick_sweep_bf16_sample(int kpad, int C);   // every SweepArgs::jt_stride-th column tile

}  // namespace gmgm_rc
