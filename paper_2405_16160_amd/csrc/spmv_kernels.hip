// Standalone CSR product y = M x for bandwidth: one short tile per workgroup
// and many workgroups resident per CU, so that the hardware keeps enough
// loads in flight to stream the matrix at HBM rate.
//
// A tile is a run of whole rows with at most kStreamNnz entries and at most
// kStreamRows rows, or a single row longer than kStreamNnz (a long tile),
// cut on the host: tiles[4 t .. 4 t + 3] = first row, end row, first entry,
// end entry.  A regular tile stages val * x[col] for all its entries in LDS
// with one burst of loads (unconditional, indices clamped into the tile),
// then sums each row with a group of lanes sized to the tile's row count
// (data-parallel-primitive lane moves, no LDS shuffles; a row far longer
// than its group is summed by a whole wave instead).  A long tile is
// summed by the whole workgroup in chunks.  Every row's sum is formed in a
// fixed order, so results are bit-reproducible.
#include "device.hpp"

namespace pdhcg {

namespace {

constexpr int kStreamBlock = 256;                          // threads per workgroup
constexpr int kStreamNnz = 2048;                           // entries per regular tile
constexpr int kStreamRows = 1024;                          // rows per regular tile
constexpr int kStreamUnroll = kStreamNnz / kStreamBlock;   // entries per thread
constexpr int kStreamRowLoads = (kStreamRows + 1 + kStreamBlock - 1) / kStreamBlock;
constexpr int kStreamWaves = kStreamBlock / kWave;

// group of lanes per row, made smaller for tiles with many rows (one pass of
// the workgroup over the tile's rows where possible)
__device__ __forceinline__ int stream_group(int mean_len, int nr) {
  int g = 1;
  while (g < mean_len && g < kWave) g <<= 1;
  const int fit = nr > 0 ? kStreamBlock / nr : kStreamBlock;
  const int f = fit >= 1 ? 1 << (31 - __clz(fit)) : 1;
  return f < g ? f : g;
}

template <typename V, typename T>
__global__ void __launch_bounds__(kStreamBlock) spmv_stream_kernel(const int32_t* __restrict__ rowptr,
                                                                   const int32_t* __restrict__ col,
                                                                   const V* __restrict__ val,
                                                                   const T* __restrict__ x, double* __restrict__ y,
                                                                   const int32_t* __restrict__ tiles) {
  __shared__ double prod[kStreamNnz];
  __shared__ int32_t rp[kStreamRows + 1];
  __shared__ double wsum[kStreamWaves];
  __shared__ int32_t wide[kStreamRows];  // rows summed by a whole wave
  __shared__ int32_t nwide;
  const int tid = threadIdx.x;
  const int32_t* t = tiles + 4 * blockIdx.x;
  const int r0 = t[0], nr = t[1] - t[0], e0 = t[2], ne = t[3] - t[2];
  if (ne > kStreamNnz) {  // one long row: chunks summed by the whole workgroup
    double s = 0.0;
    for (int base = 0; base < ne; base += kStreamNnz) {
      double part[kStreamUnroll];
#pragma unroll
      for (int u = 0; u < kStreamUnroll; ++u) {
        const int k = base + u * kStreamBlock + tid;
        const int kk = min(k, ne - 1);
        const double v = (double)gld(val + e0 + kk) * (double)gld(x + gld(col + e0 + kk));
        part[u] = k < ne ? v : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kStreamUnroll; ++u) s += part[u];
    }
    s = group_sum_last(s, kWave);
    if ((tid & (kWave - 1)) == kWave - 1) wsum[tid / kWave] = s;
    __syncthreads();
    if (tid == 0) {
      double a = wsum[0];
      for (int w = 1; w < kStreamWaves; ++w) a += wsum[w];
      gst(y + r0, a);
    }
    return;
  }
  // regular tile: row offsets and entries in one burst, then the gathers
  if (tid == 0) nwide = 0;
  int rv[kStreamRowLoads];
#pragma unroll
  for (int u = 0; u < kStreamRowLoads; ++u) rv[u] = gld(rowptr + r0 + min(u * kStreamBlock + tid, nr));
  if (ne > 0) {
    int c[kStreamUnroll];
    V v[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
      const int k = min(u * kStreamBlock + tid, ne - 1);
      c[u] = gld(col + e0 + k);
      v[u] = gld(val + e0 + k);
    }
    double g[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) g[u] = (double)gld(x + c[u]);
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
      const int k = u * kStreamBlock + tid;
      if (k < ne) prod[k] = (double)v[u] * g[u];
    }
  }
#pragma unroll
  for (int u = 0; u < kStreamRowLoads; ++u) {
    const int i = u * kStreamBlock + tid;
    if (i <= nr) rp[i] = rv[u] - e0;
  }
  __syncthreads();
  const int G = stream_group(nr > 0 ? (ne + nr - 1) / nr : 1, nr);
  const int lane = tid & (G - 1), ng = kStreamBlock / G, wlen = wide_row_len(G);
  for (int base = 0; base < nr; base += ng) {
    const int i = base + tid / G;
    const bool act = i < nr;
    const bool w = act && rp[i + 1] - rp[i] > wlen;
    double s = 0.0;
    if (act && !w) s = lane_row_sum(prod, rp[i], rp[i + 1], lane, G);
    s = group_sum_last(s, G);
    if (act && !w && lane == G - 1) gst(y + r0 + i, s);
    if (w && lane == 0) wide[atomicAdd(&nwide, 1)] = i;
  }
  __syncthreads();
  const int nw = nwide;
  const int ln = tid & (kWave - 1);
  for (int j = tid / kWave; j < nw; j += kStreamWaves) {  // wide rows: one wave each
    const int i = wide[j];
    double s = lane_row_sum(prod, rp[i], rp[i + 1], ln, kWave);
    s = group_sum_last(s, kWave);
    if (ln == kWave - 1) gst(y + r0 + i, s);
  }
}

}  // namespace

hipError_t launch_spmv_stream(const int32_t* rowptr, const int32_t* col, const double* val, const float* val32,
                              int precision, const double* x, const float* x32, double* y, const int32_t* tiles,
                              int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL((spmv_stream_kernel<float, float>), dim3(ntiles), dim3(kStreamBlock), 0, s, rowptr, col,
                       val32, x32, y, tiles);
  else
    hipLaunchKernelGGL((spmv_stream_kernel<double, double>), dim3(ntiles), dim3(kStreamBlock), 0, s, rowptr, col,
                       val, x, y, tiles);
  return hipGetLastError();
}

int spmv_stream_tile_nnz() { return kStreamNnz; }
int spmv_stream_tile_rows() { return kStreamRows; }

}  // namespace pdhcg
