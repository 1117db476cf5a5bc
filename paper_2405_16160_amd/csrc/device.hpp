// Device building blocks: NaN-propagating max, wavefront/workgroup
// reductions, a grid barrier for cooperative launches, and the row-split CSR
// row reduction used by every sparse product of the solver.
#pragma once
#include <type_traits>

#include "internal.hpp"

namespace pdhcg {
// internal linkage: the workgroup size (kBlock) differs between the
// translation units that include this header
namespace {

// max that propagates NaN (the hardware max returns the non-NaN operand, which
// would hide a diverged iterate from the termination test); written with
// selects only, so that reductions of maxima compile without branches
__device__ __forceinline__ double maxp(double a, double b) {
  const double m = a > b ? a : b;
  return (a != a || b != b) ? a + b : m;  // a + b is NaN when either is
}

// A value that every lane of the wave holds equal, marked as such for the
// compiler (it then keeps it in scalar registers instead of 64 vector lanes,
// which matters for the solver's scalar state that stays live across phases).
__device__ __forceinline__ double uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Data-parallel-primitive (DPP) lane moves of a double: each half moves with
// v_mov_b32_dpp inside the VALU, far cheaper than a shuffle through the LDS
// crossbar.  Lanes whose source lies outside the row, or whose row is masked
// off, read +0.0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Reduction over aligned groups of G lanes (G a power of two <= 64) with the
// result in the group's last lane (lane G-1 of each group): row shifts by 1,
// 2, 4, 8 make lane i hold the combination of lanes i-2^s+1 .. i of its row;
// row_bcast15 / row_bcast31 then carry row totals across the rows of a wave.
// op must have +0.0 as identity on its inputs (sums; maxima of values >= 0).
template <typename Op>
__device__ __forceinline__ double group_reduce_last(double v, int G, Op op) {
  if (G >= 2) v = op(v, dpp<0x111>(v));       // row_shr:1
  if (G >= 4) v = op(v, dpp<0x112>(v));       // row_shr:2
  if (G >= 8) v = op(v, dpp<0x114>(v));       // row_shr:4
  if (G >= 16) v = op(v, dpp<0x118>(v));      // row_shr:8
  if (G >= 32) v = op(v, dpp<0x142, 0xA>(v));  // row_bcast:15 into rows 1 and 3
  if (G >= 64) v = op(v, dpp<0x143, 0xC>(v));  // row_bcast:31 into rows 2 and 3
  return v;
}

struct AddOp {
  __device__ __forceinline__ double operator()(double a, double b) const { return a + b; }
};
struct MaxOp {
  __device__ __forceinline__ double operator()(double a, double b) const { return maxp(a, b); }
};

// sum over the aligned group of G lanes, valid in the group's last lane
__device__ __forceinline__ double group_sum_last(double v, int G) { return group_reduce_last(v, G, AddOp{}); }

// Workgroup reduction of NS sums and NM maxima at once.  Every thread ends
// with the results; the combination order is fixed, so equal inputs give
// bit-equal outputs in every workgroup.  lds must hold kWaves*(NS+NM) doubles.
template <int NS, int NM>
__device__ __forceinline__ void block_reduce(double* s, double* mx, double* lds) {
  constexpr int W = NS + NM;
#pragma unroll
  for (int k = 0; k < NS; ++k) s[k] = group_reduce_last(s[k], kWave, AddOp{});
#pragma unroll
  for (int k = 0; k < NM; ++k) mx[k] = group_reduce_last(mx[k], kWave, MaxOp{});
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == kWave - 1) {
#pragma unroll
    for (int k = 0; k < NS; ++k) lds[w * W + k] = s[k];
#pragma unroll
    for (int k = 0; k < NM; ++k) lds[w * W + NS + k] = mx[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double a = lds[k];
    for (int j = 1; j < kWaves; ++j) a += lds[j * W + k];
    s[k] = uniform(a);
  }
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    double a = lds[NS + k];
    for (int j = 1; j < kWaves; ++j) a = maxp(a, lds[j * W + NS + k]);
    mx[k] = uniform(a);
  }
  __syncthreads();
}

// Sum of per-workgroup partials part[slot*nb + j], j < nb, reduced in a
// fixed order (identical in every workgroup).  NS slots are summed, NM slots
// maximised; slots are given by index lists.
template <int NS, int NM>
__device__ __forceinline__ void reduce_partials(const double* part, int nb, const int* sum_slots,
                                                const int* max_slots, double* s, double* mx, double* lds) {
  if (nb == 1) {  // one workgroup: its own partial is the total (every thread reads it)
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] = part[sum_slots[k]];
#pragma unroll
    for (int k = 0; k < NM; ++k) mx[k] = part[max_slots[k]];
    return;
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) s[k] = 0.0;
#pragma unroll
  for (int k = 0; k < NM; ++k) mx[k] = 0.0;
  for (int j = threadIdx.x; j < nb; j += kBlock) {
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] += part[sum_slots[k] * nb + j];
#pragma unroll
    for (int k = 0; k < NM; ++k) mx[k] = maxp(mx[k], part[max_slots[k] * nb + j]);
  }
  block_reduce<NS, NM>(s, mx, lds);
}

// ------------------------------------------------------------ grid barrier
//
// Arrival is counted per XCD, in that XCD's L2: the CUs of one XCD share its
// L2, so a counter there needs no device-scope traffic.  Before arriving,
// every wave of the workgroup waits until its stores are complete (written to
// the L2); the last workgroup of an XCD to arrive then writes that L2 back to
// memory once, for the whole XCD, and arrives on the device-scope counter; the
// last XCD publishes the new generation, one copy per XCD on a line of its own.
// Waiters poll their XCD's copy with relaxed device-scope loads and take one
// acquire fence (invalidating their L1 and the XCD's L2).  The XCD of a workgroup is read from the hardware
// register that names it, and the number of the grid's workgroups on each XCD
// is counted once per launch (init), so the barrier holds for any placement of
// workgroups on XCDs.  Counters grow monotonically within a launch (64-bit),
// so no reset race exists.  Every wait is bounded by a wall-clock limit: on
// expiry the workgroup raises the abort word and returns false, and every
// other waiter then returns false too.
namespace bar {
constexpr int kMaxXcd = 16;
constexpr int kCount = 0, kAbort = kBarAbortWord, kSetup = 96;  // word offsets (256 bytes apart)
constexpr int kXcdArrive = 128;                     // + 32 x: arrivals of XCD x (in its L2)
constexpr int kXcdCount = kXcdArrive + 32 * kMaxXcd;  // + 32 x: workgroups on XCD x
constexpr int kXcdGen = kXcdCount + 32 * kMaxXcd;     // + 32 x: the generation, one copy per XCD
constexpr int kWords = kXcdGen + 32 * kMaxXcd;
static_assert(kWords <= kBarWords, "barrier words");
}  // namespace bar

#define PDHCG_LD(p) __hip_atomic_load((p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
#define PDHCG_ST(p, v) __hip_atomic_store((p), (v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
#define PDHCG_ADD(p, v) __hip_atomic_fetch_add((p), (v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)

// the XCD (accelerator complex die) this wave runs on
__device__ __forceinline__ uint32_t xcd_id() {
  uint32_t v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & (uint32_t)(bar::kMaxXcd - 1);
}

// wait until this wave's outstanding memory operations are complete (stores
// written to the L2)
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

struct GridSync {
  uint64_t* w;
  uint32_t nb;
  uint64_t epoch;
  uint32_t xcd = 0, xsize = 1, nxcd = 1;  // this workgroup's XCD, workgroups on it, XCDs in use
  static constexpr uint64_t kTimeoutTicks = 500000000ull;  // 5 s of the 100 MHz wall clock

  __device__ bool wait_word(int k, uint64_t target, int& ok) {
    const uint64_t t0 = wall_clock64();
    while (PDHCG_LD(&w[k]) < target) {
      if (PDHCG_LD(&w[bar::kAbort]) != 0ull) { ok = 0; return false; }
      if (wall_clock64() - t0 > kTimeoutTicks) {
        PDHCG_ST(&w[bar::kAbort], 1ull);
        ok = 0;
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    return true;
  }

  // Once per launch, before the first sync: count the workgroups per XCD.
  __device__ bool init() {
    __shared__ uint32_t sx[3];
    __shared__ int ok_s;
    if (threadIdx.x == 0) {
      int ok = 1;
      sx[0] = 0;
      sx[1] = 1;
      sx[2] = 1;
      if (nb > 1) {
        const uint32_t x = xcd_id();
        PDHCG_ADD(&w[bar::kXcdCount + 32 * x], 1ull);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        PDHCG_ADD(&w[bar::kSetup], 1ull);
        if (wait_word(bar::kSetup, nb, ok)) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          uint32_t used = 0;
          for (int j = 0; j < bar::kMaxXcd; ++j) used += PDHCG_LD(&w[bar::kXcdCount + 32 * j]) > 0ull;
          sx[0] = x;
          sx[1] = (uint32_t)PDHCG_LD(&w[bar::kXcdCount + 32 * x]);
          sx[2] = used;
        }
      }
      ok_s = ok;
    }
    __syncthreads();
    xcd = sx[0];
    xsize = sx[1];
    nxcd = sx[2];
    return ok_s != 0;
  }

  __device__ bool sync() {
    __shared__ int ok_s;
    if (nb > 1) wait_stores();
    __syncthreads();
    ++epoch;
    if (threadIdx.x == 0) {
      int ok = 1;
      if (nb > 1) {
        const uint64_t a = __hip_atomic_fetch_add(&w[bar::kXcdArrive + 32 * xcd], 1ull, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
        if (a == (uint64_t)xsize * epoch - 1) {  // last of its XCD: write the XCD's L2 back once
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          const uint64_t t = PDHCG_ADD(&w[bar::kCount], 1ull);
          if (t == (uint64_t)nxcd * epoch - 1) {  // publish to every XCD's own line
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            for (int x = 0; x < bar::kMaxXcd; ++x) PDHCG_ST(&w[bar::kXcdGen + 32 * x], epoch);
          }
        }
        wait_word(bar::kXcdGen + 32 * xcd, epoch, ok);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0;
  }
};

// ------------------------------------------------------- row-split products

// Value loaders: FP64 or FP32 matrix values, FP64 or FP32 gathered vectors;
// products are accumulated in FP64.
template <typename V>
__device__ __forceinline__ double ldv(const V* p, int k) { return (double)p[k]; }

// Load through a global-address-space pointer (the solver's arrays all live
// in device memory; a generic pointer would make the compiler emit flat loads,
// which also count against the LDS counter and force wider waits).
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// The same with the non-temporal hint, for a matrix streamed once per
// product: its lines should not displace the reused vectors and index data
// (of this workgroup and of the others on the XCD) from the L2 and the MALL.
template <typename T>
__device__ __forceinline__ T gld_nt(const T* p) {
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}

// Four consecutive FP32 values from a 4-byte aligned address in one
// global_load_dwordx4 (gfx950 takes dword-aligned 16-byte accesses), plain
// or with the non-temporal hint.
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ f32x4u gld4(const float* p) {
  return *(const __attribute__((address_space(1))) f32x4u*)p;
}
__device__ __forceinline__ f32x4u gld4_nt(const float* p) {
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) f32x4u*)p);
}

// an (r, p) record of the textbook CG: one 8-byte load or store
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f32x2 gld2(const float2* p) {
  return *(const __attribute__((address_space(1))) f32x2*)p;
}
__device__ __forceinline__ void gst2(float2* p, float a, float b) {
  *(__attribute__((address_space(1))) f32x2*)p = f32x2{a, b};
}

template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

// float4 rows move as one 16-byte access (through the clang vector type: the
// HIP vector class has no constructors for address-space-qualified operands)
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <>
__device__ __forceinline__ float4 gld<float4>(const float4* p) {
  const f32x4 v = *(const __attribute__((address_space(1))) f32x4*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}

template <>
__device__ __forceinline__ void gst<float4>(float4* p, float4 v) {
  f32x4 w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  *(__attribute__((address_space(1))) f32x4*)p = w;
}

// sum_k M[i,k] * g(col[k]) for the entries [beg, end) of one row, computed by
// `width` lanes starting at lane `lane` (partial sums; reduced by the caller)
// Loads go in batches of 8 per lane, unconditional (indices clamped into the
// row): 8 index/value loads, then 8 gathers, instead of one dependent pair at
// a time.
template <typename V, typename Gather>
__device__ __forceinline__ double row_partial(const int32_t* col, const V* val, int beg, int end, int lane,
                                              int width, const Gather& g) {
  constexpr int U = 8;
  double s = 0.0;
  for (int base = beg + lane; base < end; base += U * width) {
    int c[U];
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = min(base + u * width, end - 1);
      c[u] = gld(col + k);
      v[u] = gld(val + k);
    }
    double gv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) gv[u] = g(c[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (base + u * width < end) s += (double)v[u] * gv[u];
  }
  return s;
}

template <typename T>
struct GatherVec {
  const T* v;
  __device__ __forceinline__ double operator()(int j) const { return (double)gld(v + j); }
};

// p_j = r_j + beta p_prev_j, formed at gather time (the CG direction update is
// folded into the next product, which saves a grid barrier per CG step)
template <typename T>
struct GatherDir {
  const T* r;
  const T* pp;
  double beta;
  int first;
  // both loads are unconditional (pp is always a valid buffer; when first is
  // set its contents are not used), so a tile's gathers issue together
  __device__ __forceinline__ double operator()(int j) const {
    const double rj = (double)gld(r + j), pj = (double)gld(pp + j);
    return first ? rj : rj + beta * pj;
  }
};

// The same from the interleaved FP32 records (r_j, p_prev_j): one 8-byte
// load, one cache line, per gathered entry
struct GatherDir2 {
  const float2* rp;
  double beta;
  int first;
  __device__ __forceinline__ double operator()(int j) const {
    const f32x2 w = gld2(rp + j);
    const double rj = (double)w.x, pj = (double)w.y;
    return first ? rj : rj + beta * pj;
  }
};

// ----------------------------------------------------- LDS-staged tiles

struct TileLds {
  double prod[kTileNnz];
  double sum1[kTileRows];
  double sum2[kTileRows];
  int32_t rp[kTileRows + 1];
  int32_t rp2[kTileRows + 1];
  int32_t wide[kTileRows];  // rows of the tile summed by a whole wave
  int32_t nwide;
};

// the workgroup's single LDS staging area for tiles
__device__ __forceinline__ TileLds& tile_lds() {
  __shared__ TileLds L;
  return L;
}

constexpr int kStageUnroll = kTileNnz / kBlock;  // entries per thread: one burst per tile
constexpr int kRowsPerThread = (kTileRows + 1 + kBlock - 1) / kBlock;

// Stage one tile in LDS with every load of the tile in flight at once:
// row offsets of up to two matrices (rp1, rp2: rowptr[ra + i] - base), and the
// entry list [M1 entries z0..z0+nz, M2 entries w0..w0+nw] as products
// val * g(col) into prod[0 .. nz+nw).  Every load is unconditional (indices
// are clamped into the tile, surplus lanes repeat the last entry and store
// nothing), so the index, value and row-pointer loads all issue before the
// first wait, then all gathers before the next.
template <typename V, typename G1, typename G2>
__device__ __forceinline__ void stage_tile(const int32_t* rowptr1, const int32_t* col1, const V* val1, const G1& g1,
                                           int z0, int nz, const int32_t* rowptr2, const int32_t* col2,
                                           const V* val2, const G2& g2, int w0, int nw, int ra, int nr,
                                           int32_t* rp1, int32_t* rp2, double* prod) {
  const int tid = threadIdx.x;
  int r1[kRowsPerThread], r2[kRowsPerThread];
#pragma unroll
  for (int u = 0; u < kRowsPerThread; ++u) {
    const int i = min(u * kBlock + tid, nr);
    r1[u] = rowptr1 ? gld(rowptr1 + ra + i) : 0;
    r2[u] = rowptr2 ? gld(rowptr2 + ra + i) : 0;
  }
  const int ntot = nz + nw;
  if (ntot > 0) {
    int c[kStageUnroll];
    V v[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int k = min(u * kBlock + tid, ntot - 1);
      const bool first = k < nz;
      c[u] = gld(first ? col1 + z0 + k : col2 + w0 + (k - nz));
      v[u] = gld(first ? val1 + z0 + k : val2 + w0 + (k - nz));
    }
    double gv[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int k = min(u * kBlock + tid, ntot - 1);
      if constexpr (std::is_same<G1, G2>::value) {
        const G1 g = k < nz ? g1 : g2;
        gv[u] = g(c[u]);
      } else {
        gv[u] = k < nz ? g1(c[u]) : g2(c[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int k = u * kBlock + tid;
      if (k < ntot) prod[k] = (double)v[u] * gv[u];
    }
  }
#pragma unroll
  for (int u = 0; u < kRowsPerThread; ++u) {
    const int i = u * kBlock + tid;
    if (i <= nr) {
      if (rowptr1) rp1[i] = r1[u] - z0;
      if (rowptr2) rp2[i] = r2[u] - w0 + nz;
    }
  }
}

// Lanes per row for a tile's row sums: the partition's group size G, made
// smaller when the tile has many rows, so that all of its rows are summed in
// one pass of the workgroup (two when it has more rows than threads); each
// lane then adds a longer stretch of the row.
__device__ __forceinline__ int tile_group(int G, int nr) {
  const int fit = nr > 0 ? kBlock / nr : kBlock;
  const int g = fit >= 1 ? 1 << (31 - __clz(fit)) : 1;
  return g < G ? g : G;
}

// A row longer than this many entries per lane of its group is summed by a
// whole wave instead (skewed tiles: one long row among many short ones)
constexpr int kLaneEntries = 8;
__device__ __forceinline__ int wide_row_len(int G) { return kLaneEntries * G > kWave ? kLaneEntries * G : kWave; }

// sum of prod[k] for k = beg + lane, beg + lane + G, ... < end (two chains)
__device__ __forceinline__ double lane_row_sum(const double* prod, int beg, int end, int lane, int G) {
  double a0 = 0.0, a1 = 0.0;
  int k = beg + lane;
  for (; k + G < end; k += 2 * G) {
    a0 += prod[k];
    a1 += prod[k + G];
  }
  if (k < end) a0 += prod[k];
  return a0 + a1;
}

constexpr int kEpiRows = kTileRows / kBlock;  // epilogue rows per thread in one tile
static_assert(kTileRows % kBlock == 0, "tile rows split evenly over the threads");

// The no-op prefetch of tile_rows / tile_rows2.
struct NoPre {
  __device__ __forceinline__ int operator()(int) const { return 0; }
};

// Load through a pointer known to address LDS (ds_read rather than a flat load)
template <typename T>
__device__ __forceinline__ T lld(const T* p) {
  return *(const __attribute__((address_space(3))) T*)p;
}

// store through a generic pointer known to point into LDS
template <typename T>
__device__ __forceinline__ void lst(T* p, T v) {
  *(__attribute__((address_space(3))) T*)p = v;
}

// Stage one tile of a single matrix whose rows of the workgroup are held in
// LDS (lrp[j] = rowptr[roff + j]; lcol / lval hold the entries from eoff):
// the same products as stage_tile, with only the gathers going to memory.
template <typename V, typename G1>
__device__ __forceinline__ void stage_tile_lds(const int32_t* lrp, int roff, const int32_t* lcol, const V* lval,
                                               int eoff, const G1& g, int z0, int nz, int ra, int nr, int32_t* rp1,
                                               double* prod) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kRowsPerThread; ++u) {
    const int i = u * kBlock + tid;
    if (i <= nr) rp1[i] = lld(lrp + ra + i - roff) - z0;
  }
  if (nz > 0) {
    int c[kStageUnroll];
    V v[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int k = z0 - eoff + min(u * kBlock + tid, nz - 1);
      c[u] = lld(lcol + k);
      v[u] = lld(lval + k);
    }
    double gv[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) gv[u] = g(c[u]);
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int k = u * kBlock + tid;
      if (k < nz) prod[k] = (double)v[u] * gv[u];
    }
  }
}

// One tile of a single matrix.  pre(row) loads the row epilogue's own inputs
// (rows of the tile, indices clamped into it) and is issued together with the
// tile's staging loads, so those inputs cost no extra memory round trip.  Row
// sums are formed by G-lane groups from the staged products and parked in LDS;
// then epi(row, sum, pre(row)) runs with one thread per row.
// stage(L, ra, nr, z0, nz) fills L.rp and L.prod for the tile
template <typename Stage, typename Pre, typename Epi>
__device__ __forceinline__ void tile_rows_impl(const int32_t* t, int G, const Stage& stage, const Pre& pre,
                                               Epi epi) {
  TileLds& L = tile_lds();
  const int ra = t[0], nr = t[1] - t[0], z0 = t[2], nz = t[3] - t[2];
  using PV = decltype(pre(0));
  PV pv[kEpiRows];
  if (nr > 0) {
#pragma unroll
    for (int u = 0; u < kEpiRows; ++u) pv[u] = pre(ra + min(u * kBlock + (int)threadIdx.x, nr - 1));
  }
  if (threadIdx.x == 0) L.nwide = 0;
  stage(L, ra, nr, z0, nz);
  __syncthreads();
  const int Gt = tile_group(G, nr);
  const int lane = threadIdx.x & (Gt - 1), ng = kBlock / Gt, wlen = wide_row_len(Gt);
  for (int base = 0; base < nr; base += ng) {
    const int i = base + (int)threadIdx.x / Gt;
    const bool act = i < nr;
    const bool wide = act && L.rp[i + 1] - L.rp[i] > wlen;
    double s = 0.0;
    if (act && !wide) s = lane_row_sum(L.prod, L.rp[i], L.rp[i + 1], lane, Gt);
    s = group_sum_last(s, Gt);
    if (act && !wide && lane == Gt - 1) L.sum1[i] = s;
    if (wide && lane == 0) L.wide[atomicAdd(&L.nwide, 1)] = i;
  }
  __syncthreads();
  const int nw = L.nwide;
  if (nw > 0) {  // wide rows: one wave each
    const int ln = threadIdx.x & (kWave - 1);
    for (int j = (int)threadIdx.x / kWave; j < nw; j += kWaves) {
      const int i = L.wide[j];
      double s = lane_row_sum(L.prod, L.rp[i], L.rp[i + 1], ln, kWave);
      s = group_sum_last(s, kWave);
      if (ln == kWave - 1) L.sum1[i] = s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < kEpiRows; ++u) {
    const int i = u * kBlock + (int)threadIdx.x;
    if (i < nr) epi(ra + i, L.sum1[i], pv[u]);
  }
  __syncthreads();
}

template <typename V, typename Gather, typename Pre, typename Epi>
__device__ __forceinline__ void tile_rows_pf(const int32_t* rowptr, const int32_t* col, const V* val,
                                             const int32_t* t, int G, const Gather& g, const Pre& pre, Epi epi) {
  tile_rows_impl(
      t, G,
      [&](TileLds& L, int ra, int nr, int z0, int nz) {
        stage_tile(rowptr, col, val, g, z0, nz, (const int32_t*)nullptr, col, val, g, z0, 0, ra, nr, L.rp, L.rp2,
                   L.prod);
      },
      pre, epi);
}

// the same over the workgroup's rows held in LDS (see stage_tile_lds)
template <typename V, typename Gather, typename Pre, typename Epi>
__device__ __forceinline__ void tile_rows_res(const int32_t* lrp, int roff, const int32_t* lcol, const V* lval,
                                              int eoff, const int32_t* t, int G, const Gather& g, const Pre& pre,
                                              Epi epi) {
  tile_rows_impl(
      t, G,
      [&](TileLds& L, int ra, int nr, int z0, int nz) {
        stage_tile_lds(lrp, roff, lcol, lval, eoff, g, z0, nz, ra, nr, L.rp, L.prod);
      },
      pre, epi);
}

template <typename V, typename Gather, typename Epi>
__device__ __forceinline__ void tile_rows(const int32_t* rowptr, const int32_t* col, const V* val, const int32_t* t,
                                          int G, const Gather& g, Epi epi) {
  tile_rows_pf(rowptr, col, val, t, G, g, NoPre{}, [&](int i, double s, int) { epi(i, s); });
}

// One tile of two matrices over the same rows (the stacked [Q | A'] pass):
// epi(row, sum1, sum2, pre(row)).  M2 may be absent (rowptr2 == nullptr: sum2 = 0).
template <typename Gather1, typename Gather2, typename Pre, typename Epi>
__device__ __forceinline__ void tile_rows2(const int32_t* rowptr1, const int32_t* col1, const double* val1,
                                           const Gather1& g1, const int32_t* rowptr2, const int32_t* col2,
                                           const double* val2, const Gather2& g2, const int32_t* t, int G,
                                           const Pre& pre, Epi epi) {
  TileLds& L = tile_lds();
  const int ra = t[0], nr = t[1] - t[0];
  const int z0 = t[2], nz = rowptr1 ? t[3] - t[2] : 0, w0 = t[4], nw = rowptr2 ? t[5] - t[4] : 0;
  using PV = decltype(pre(0));
  PV pv[kEpiRows];
  if (nr > 0) {
#pragma unroll
    for (int u = 0; u < kEpiRows; ++u) pv[u] = pre(ra + min(u * kBlock + (int)threadIdx.x, nr - 1));
  }
  if (threadIdx.x == 0) L.nwide = 0;
  stage_tile(rowptr1, col1, val1, g1, z0, nz, rowptr2, col2, val2, g2, w0, nw, ra, nr, L.rp, L.rp2, L.prod);
  __syncthreads();
  const int Gt = tile_group(G, nr);
  const int lane = threadIdx.x & (Gt - 1), ng = kBlock / Gt, wlen = wide_row_len(Gt);
  auto len1 = [&](int i) { return rowptr1 ? L.rp[i + 1] - L.rp[i] : 0; };
  auto len2 = [&](int i) { return rowptr2 ? L.rp2[i + 1] - L.rp2[i] : 0; };
  for (int base = 0; base < nr; base += ng) {
    const int i = base + (int)threadIdx.x / Gt;
    const bool act = i < nr;
    const bool wide = act && (len1(i) > wlen || len2(i) > wlen);
    double s1 = 0.0, s2 = 0.0;
    if (act && !wide) {
      if (rowptr1) s1 = lane_row_sum(L.prod, L.rp[i], L.rp[i + 1], lane, Gt);
      if (rowptr2) s2 = lane_row_sum(L.prod, L.rp2[i], L.rp2[i + 1], lane, Gt);
    }
    s1 = group_sum_last(s1, Gt);
    s2 = group_sum_last(s2, Gt);
    if (act && !wide && lane == Gt - 1) {
      L.sum1[i] = s1;
      L.sum2[i] = s2;
    }
    if (wide && lane == 0) L.wide[atomicAdd(&L.nwide, 1)] = i;
  }
  __syncthreads();
  const int nwr = L.nwide;
  if (nwr > 0) {  // wide rows: one wave each
    const int ln = threadIdx.x & (kWave - 1);
    for (int j = (int)threadIdx.x / kWave; j < nwr; j += kWaves) {
      const int i = L.wide[j];
      double s1 = 0.0, s2 = 0.0;
      if (rowptr1) s1 = lane_row_sum(L.prod, L.rp[i], L.rp[i + 1], ln, kWave);
      if (rowptr2) s2 = lane_row_sum(L.prod, L.rp2[i], L.rp2[i + 1], ln, kWave);
      s1 = group_sum_last(s1, kWave);
      s2 = group_sum_last(s2, kWave);
      if (ln == kWave - 1) {
        L.sum1[i] = s1;
        L.sum2[i] = s2;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < kEpiRows; ++u) {
    const int i = u * kBlock + (int)threadIdx.x;
    if (i < nr) epi(ra + i, L.sum1[i], L.sum2[i], pv[u]);
  }
  __syncthreads();
}

}  // namespace
}  // namespace pdhcg
