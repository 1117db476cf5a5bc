// Warm-start network on the GPU: bfloat16 matrix products on MFMA with FP32
// accumulation, fused bias / ReLU / ReLU-derivative epilogues, MSE gradient,
// bias-gradient column sums and Adam on FP32 master weights.  Host side of
// include/pdhcg_mlp.h at the end of the file.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/pdhcg.h"
#include "../../include/pdhcg_mlp.h"
#include "internal.hpp"

namespace pdhcg {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest, ties to even (NaN kept quiet)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

constexpr int GB = 64;   // block tile (rows and columns)
constexpr int GK = 32;   // k per LDS stage (one K = 32 MFMA step)
constexpr int GP = 8;    // LDS row padding (bf16 elements; rows stay 16-byte aligned)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// Stage an R x C tile of a strided bf16 matrix M(r, c) = M[r*sr + c*sc]
// (rows r0.., columns c0.., bounds nr, nc; zeros outside) into T[R][C + GP],
// 8 elements per thread.  Along a unit stride the 8 elements are one 16-byte
// load when they are in range and aligned; otherwise they are loaded one by
// one.  Unit stride along c: the 8 land in one row (one 16-byte LDS store);
// along r: in 8 rows of one column.
template <int R, int C>
__device__ __forceinline__ void stage_bf16(uint16_t (*T)[C + GP], const uint16_t* __restrict__ M, int64_t sr,
                                           int64_t sc, int r0, int c0, int nr, int nc) {
  static_assert(R * C == 8 * 256, "one 8-element vector per thread");
  const int tid = threadIdx.x;
  if (sc == 1) {  // contiguous along c: thread -> (row, 8 columns)
    const int r = tid / (C / 8), c = (tid % (C / 8)) * 8;
    const int gr = r0 + r, gc = c0 + c;
    const int64_t off = (int64_t)gr * sr + gc;
    u16x8 v;
    if (gr < nr && gc + 8 <= nc && (off & 7) == 0) {
      v = *reinterpret_cast<const u16x8*>(M + off);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (gr < nr && gc + e < nc) ? M[off + e] : (uint16_t)0;
    }
    *reinterpret_cast<u16x8*>(&T[r][c]) = v;
  } else if (sr == 1) {  // contiguous along r: thread -> (8 rows, column)
    const int c = tid / (R / 8), r = (tid % (R / 8)) * 8;
    const int gr = r0 + r, gc = c0 + c;
    const int64_t off = gr + (int64_t)gc * sc;
    u16x8 v;
    if (gc < nc && gr + 8 <= nr && (off & 7) == 0) {
      v = *reinterpret_cast<const u16x8*>(M + off);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (gc < nc && gr + e < nr) ? M[off + e] : (uint16_t)0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) T[r + e][c] = v[e];
  } else {  // general strides
    const int r = tid / (C / 8), c = (tid % (C / 8)) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int gr = r0 + r, gc = c0 + c + e;
      T[r][c + e] = (gr < nr && gc < nc) ? M[(int64_t)gr * sr + (int64_t)gc * sc] : (uint16_t)0;
    }
  }
}

// C = A B on bfloat16 operands with FP32 accumulation.  A(m,k) = A[m*sam +
// k*sak], B(k,n) = B[k*sbk + n*sbn], so transposed operands need no copy.
// Each of the four waves owns a 32 x 32 quarter of the 64 x 64 block tile as
// 2 x 2 tiles of the gfx950 MFMA 16x16x32 (eight bfloat16 per lane and
// operand); a 32-deep k stage of A and of B (kept n-major) sits in LDS.
// Epilogue: + bias[n]; ReLU; zero where mask(m,n) <= 0 (ReLU derivative);
// FP32 and/or bfloat16 output.  With Cpart set, workgroup z of the grid's z
// dimension takes k in [z kchunk, (z + 1) kchunk) and writes its raw partial
// product to Cpart[z][m][n] (M x N), summed by splitk_finish (split-K for
// products with few output tiles and a long k).
__device__ __forceinline__ float gemm_epilogue(float v, int m, int n, const float* __restrict__ bias, int relu,
                                               const uint16_t* __restrict__ mask, int64_t ldc) {
  if (bias) v += bias[n];
  if (relu) v = v > 0.f ? v : 0.f;
  if (mask && !(from_bf16(mask[(int64_t)m * ldc + n]) > 0.f)) v = 0.f;
  return v;
}

__global__ void __launch_bounds__(256) gemm_bf16(int M, int N, int K, const uint16_t* __restrict__ A, int64_t sam,
                                                 int64_t sak, const uint16_t* __restrict__ Bm, int64_t sbk,
                                                 int64_t sbn, const float* __restrict__ bias, int relu,
                                                 const uint16_t* __restrict__ mask, float* __restrict__ Cf,
                                                 uint16_t* __restrict__ Cb, int64_t ldc, int kchunk,
                                                 float* __restrict__ Cpart) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GB][GK + GP];
  __shared__ __attribute__((aligned(16))) uint16_t Bt[GB][GK + GP];  // B tile stored as [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * GB, n0 = blockIdx.x * GB;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  for (int k0 = kb; k0 < ke; k0 += GK) {
    stage_bf16<GB, GK>(As, A, sam, sak, m0, k0, M, ke);    // As[m][k]
    stage_bf16<GB, GK>(Bt, Bm, sbn, sbk, n0, k0, N, ke);   // Bt[n][k] = B(k, n)
    __syncthreads();
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(&Bt[wn * 32 + j * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m < M && n < N) {
          if (Cpart) {
            Cpart[((int64_t)blockIdx.z * M + m) * N + n] = acc[i][j][r];
            continue;
          }
          const float v = gemm_epilogue(acc[i][j][r], m, n, bias, relu, mask, ldc);
          if (Cf) Cf[(int64_t)m * ldc + n] = v;
          if (Cb) Cb[(int64_t)m * ldc + n] = to_bf16(v);
        }
      }
}

// sum of the split-K partials in order z = 0 .. S-1, then the epilogue
__global__ void splitk_finish(const float* __restrict__ Cpart, int S, int M, int N, const float* __restrict__ bias,
                              int relu, const uint16_t* __restrict__ mask, float* __restrict__ Cf,
                              uint16_t* __restrict__ Cb, int64_t ldc) {
  const int64_t mn = (int64_t)M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < mn; e += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    for (int z = 0; z < S; ++z) v += Cpart[z * mn + e];
    const int m = (int)(e / N), n = (int)(e - (int64_t)m * N);
    v = gemm_epilogue(v, m, n, bias, relu, mask, ldc);
    if (Cf) Cf[(int64_t)m * ldc + n] = v;
    if (Cb) Cb[(int64_t)m * ldc + n] = to_bf16(v);
  }
}

__global__ void f32_to_bf16(const float* __restrict__ in, uint16_t* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = to_bf16(in[i]);
}

// out (batch x cols, bfloat16) = rows rows[0..batch) of in (FP32, cols per row)
__global__ void rows_to_bf16(const float* __restrict__ in, const int32_t* __restrict__ rows, int batch, int cols,
                             uint16_t* __restrict__ out) {
  const int64_t n = (int64_t)batch * cols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i - r * cols;
    out[i] = to_bf16(in[(int64_t)rows[r] * cols + c]);
  }
}

// G = 2 (O - T) / count (FP32 and bfloat16 copies); per-block partial sums of
// (O - T)^2.  Row r of T is T's row rows[r] when rows is given (cols per row).
__global__ void mse_grad(const float* __restrict__ O, const float* __restrict__ T, const int32_t* __restrict__ rows,
                         int cols, int64_t n, float scale, float* __restrict__ G, uint16_t* __restrict__ Gb,
                         double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t ti = i;
    if (rows) {
      const int64_t r = i / cols;
      ti = (int64_t)rows[r] * cols + (i - r * cols);
    }
    const float d = O[i] - T[ti];
    s += (double)d * (double)d;
    const float g = 2.0f * d * scale;
    G[i] = g;
    Gb[i] = to_bf16(g);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// the loss of a step, and its running sum over the training steps (acc[0])
// with their count (acc[1])
// (one workgroup of 256 threads: strided partial sums, then a fixed-order tree)
__global__ void __launch_bounds__(256) sum_partials(const double* __restrict__ partial, int n, double scale,
                                                    float* __restrict__ out, double* __restrict__ acc) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double t = red[0] * scale;
    *out = (float)t;
    acc[0] += t;
    acc[1] += 1.0;
  }
}

// out[c] = sum_r M[r, c] (bias gradients): a workgroup takes 16 columns, its
// 16 row groups sum rows g, g + 16, ... and the groups' sums are added in a
// fixed order
constexpr int CS_COLS = 16, CS_GROUPS = 16;
__global__ void __launch_bounds__(CS_COLS * CS_GROUPS) colsum(const float* __restrict__ Mx, int rows, int cols,
                                                             float* __restrict__ out) {
  __shared__ float part[CS_GROUPS][CS_COLS];
  const int cl = threadIdx.x % CS_COLS, g = threadIdx.x / CS_COLS;
  const int c = blockIdx.x * CS_COLS + cl;
  float s = 0.f;
  if (c < cols)
    for (int r = g; r < rows; r += CS_GROUPS) s += Mx[(int64_t)r * cols + c];
  part[g][cl] = s;
  __syncthreads();
  if (g == 0 && c < cols) {
    float t = part[0][cl];
    for (int k = 1; k < CS_GROUPS; ++k) t += part[k][cl];
    out[c] = t;
  }
}

// Adam on FP32 masters; refreshes the bfloat16 copy where wb != null
__global__ void adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                     int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                     uint16_t* __restrict__ wb) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = to_bf16(wi);
  }
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 2048) g = 2048;
  return (int)g;
}

// The network's outputs of `rows` rows (Z, FP32, n_out per row) turned into a
// start point, rows r0 .. r0 + rows of the packed x0 (n per row) and y0 (m per
// row): column c < n gives x_c = z_c sd_c + mu_c; column n + p (p < n_pair)
// the multiplier lam of the p-th equality pair, y[plus_p] = max(lam, 0) and
// y[minus_p] = max(-lam, 0); column n + n_pair + q gives y[rest_q] =
// max(v, 0).  The product and the sum are rounded separately (contraction
// into a fused multiply-add is switched off here), as a host computation of
// the same formula does.
__global__ void decode_start(const float* __restrict__ Z, int rows, int n_out, const double* __restrict__ mu,
                             const double* __restrict__ sd, int n, int n_pair, const int32_t* __restrict__ plus,
                             const int32_t* __restrict__ minus, const int32_t* __restrict__ rest, int m, int64_t r0,
                             double* __restrict__ x0, double* __restrict__ y0) {
#pragma clang fp contract(off)
  const int64_t total = (int64_t)rows * n_out;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n_out;
    const int c = (int)(e - r * n_out);
    const double v = (double)Z[e] * sd[c] + mu[c];
    const int64_t row = r0 + r;
    if (c < n) {
      x0[row * n + c] = v;
    } else if (c < n + n_pair) {
      const int p = c - n;
      y0[row * m + plus[p]] = v > 0.0 ? v : 0.0;
      y0[row * m + minus[p]] = -v > 0.0 ? -v : 0.0;
    } else {
      y0[row * m + rest[c - n - n_pair]] = v > 0.0 ? v : 0.0;
    }
  }
}

}  // namespace
}  // namespace pdhcg

using namespace pdhcg;

struct pdhcg_mlp {
  int n_in = 0, n_hid = 0, n_out = 0, cap = 0;
  hipStream_t stream = nullptr;
  int64_t np = 0;
  int64_t off[6] = {0, 0, 0, 0, 0, 0};  // W1 b1 W2 b2 W3 b3 in the packed vector
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* wb = nullptr;               // bfloat16 copy of the packed vector (weights used)
  int64_t t = 0;
  uint16_t *xb = nullptr, *h1 = nullptr, *h2 = nullptr, *gob = nullptr, *d2b = nullptr, *d1b = nullptr;
  float *out = nullptr, *go = nullptr, *d2 = nullptr, *d1 = nullptr, *loss = nullptr;
  double* partial = nullptr;
  double* loss_acc = nullptr;  // [sum of step losses, steps] since the last pdhcg_mlp_take_loss
  float* kpart = nullptr;      // split-K partial products (kSplitMax x kSplitTiles block tiles)
  std::vector<void*> allocs;
  ~pdhcg_mlp() {
    for (void* p : allocs) (void)hipFree(p);
  }
  template <typename T>
  bool alloc(T** p, int64_t count) {
    if (hipMalloc((void**)p, sizeof(T) * (size_t)(count > 0 ? count : 1)) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    allocs.push_back(*p);
    return true;
  }
};

namespace {

#define MLPX(call)                                                                                  \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return set_error(PDHCG_ERR_HIP, (std::string(#call) + ": " + hipGetErrorString(e_)).c_str()); \
  } while (0)

// A product with fewer output tiles than this and k >= 512 is split along k
// (at most kSplitMax parts of >= 256 k each) so that more CUs take part.
constexpr int kSplitTiles = 128, kSplitMax = 8;

hipError_t gemm(hipStream_t s, float* work, int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak,
                const uint16_t* B, int64_t sbk, int64_t sbn, const float* bias, int relu, const uint16_t* mask,
                float* Cf, uint16_t* Cb, int64_t ldc) {
  const int gx = (N + GB - 1) / GB, gy = (M + GB - 1) / GB;
  int S = 1, kchunk = K;
  if (work && gx * gy < kSplitTiles && K >= 512) {
    S = std::min(std::min(kSplitMax, (2 * kSplitTiles + gx * gy - 1) / (gx * gy)), K / 256);
    kchunk = ((K + S - 1) / S + GK - 1) / GK * GK;
    S = (K + kchunk - 1) / kchunk;
  }
  if (S <= 1) {
    hipLaunchKernelGGL(gemm_bf16, dim3(gx, gy, 1), dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, bias, relu,
                       mask, Cf, Cb, ldc, K, (float*)nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(gemm_bf16, dim3(gx, gy, S), dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, bias, relu,
                     mask, Cf, Cb, ldc, kchunk, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t mn = (int64_t)M * N;
  hipLaunchKernelGGL(splitk_finish, dim3((int)std::min<int64_t>((mn + 255) / 256, 2048)), dim3(256), 0, s, work, S, M,
                     N, bias, relu, mask, Cf, Cb, ldc);
  return hipGetLastError();
}

int check_batch(const pdhcg_mlp* h, int32_t batch) {
  if (!h) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null network handle");
  if (batch < 1 || batch > h->cap) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "batch outside 1..max_batch");
  return 0;
}

// forward pass of `batch` rows of X (device FP32: the first batch rows, or
// rows[0..batch) when rows is given) into h->out; keeps the bfloat16
// activations for the backward pass
int run_forward(pdhcg_mlp* h, const float* X, const int32_t* rows, int batch) {
  const int a = h->n_in, d = h->n_hid, o = h->n_out;
  if (rows)
    hipLaunchKernelGGL(rows_to_bf16, dim3(grid_for((int64_t)batch * a)), dim3(256), 0, h->stream, X, rows, batch, a,
                       h->xb);
  else
    hipLaunchKernelGGL(f32_to_bf16, dim3(grid_for((int64_t)batch * a)), dim3(256), 0, h->stream, X, h->xb,
                       (int64_t)batch * a);
  MLPX(hipGetLastError());
  MLPX(gemm(h->stream, h->kpart, batch, d, a, h->xb, a, 1, h->wb + h->off[0], d, 1, h->w + h->off[1], 1, nullptr, nullptr, h->h1,
            d));
  MLPX(gemm(h->stream, h->kpart, batch, d, d, h->h1, d, 1, h->wb + h->off[2], d, 1, h->w + h->off[3], 1, nullptr, nullptr, h->h2,
            d));
  MLPX(gemm(h->stream, h->kpart, batch, o, d, h->h2, d, 1, h->wb + h->off[4], o, 1, h->w + h->off[5], 0, nullptr, h->out,
            nullptr, o));
  return 0;
}

// forward pass, MSE gradient and backward pass of one batch, queued on the
// network's stream (no wait); the gradient stays in h->g, the loss in h->loss
int queue_loss_grad(pdhcg_mlp* h, const float* X, const float* T, const int32_t* rows, int batch) {
  int rc;
  if ((rc = run_forward(h, X, rows, batch))) return rc;
  const int a = h->n_in, d = h->n_hid, o = h->n_out;
  const int64_t no = (int64_t)batch * o;
  const int pg = 512;
  hipLaunchKernelGGL(mse_grad, dim3(pg), dim3(256), 0, h->stream, h->out, T, rows, o, no, (float)(1.0 / (double)no),
                     h->go, h->gob, h->partial);
  MLPX(hipGetLastError());
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, h->stream, h->partial, pg, 1.0 / (double)no, h->loss,
                     h->loss_acc);
  MLPX(hipGetLastError());
  float* g = h->g;
  // layer 3: dW3 = H2' G, db3 = colsum G, dH2 = (G W3') masked by H2 > 0
  MLPX(gemm(h->stream, h->kpart, d, o, batch, h->h2, 1, d, h->gob, o, 1, nullptr, 0, nullptr, g + h->off[4], nullptr, o));
  hipLaunchKernelGGL(colsum, dim3((o + CS_COLS - 1) / CS_COLS), dim3(CS_COLS * CS_GROUPS), 0, h->stream, h->go, batch,
                     o, g + h->off[5]);
  MLPX(hipGetLastError());
  MLPX(gemm(h->stream, h->kpart, batch, d, o, h->gob, o, 1, h->wb + h->off[4], 1, o, nullptr, 0, h->h2, h->d2, h->d2b, d));
  // layer 2
  MLPX(gemm(h->stream, h->kpart, d, d, batch, h->h1, 1, d, h->d2b, d, 1, nullptr, 0, nullptr, g + h->off[2], nullptr, d));
  hipLaunchKernelGGL(colsum, dim3((d + CS_COLS - 1) / CS_COLS), dim3(CS_COLS * CS_GROUPS), 0, h->stream, h->d2, batch,
                     d, g + h->off[3]);
  MLPX(hipGetLastError());
  MLPX(gemm(h->stream, h->kpart, batch, d, d, h->d2b, d, 1, h->wb + h->off[2], 1, d, nullptr, 0, h->h1, h->d1, h->d1b, d));
  // layer 1
  MLPX(gemm(h->stream, h->kpart, a, d, batch, h->xb, 1, a, h->d1b, d, 1, nullptr, 0, nullptr, g + h->off[0], nullptr, d));
  hipLaunchKernelGGL(colsum, dim3((d + CS_COLS - 1) / CS_COLS), dim3(CS_COLS * CS_GROUPS), 0, h->stream, h->d1, batch,
                     d, g + h->off[1]);
  MLPX(hipGetLastError());
  return 0;
}

int queue_adam(pdhcg_mlp* h, float lr, float beta1, float beta2, float eps) {
  h->t += 1;
  const float c1 = (float)(1.0 - pow((double)beta1, (double)h->t));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)h->t));
  hipLaunchKernelGGL(adam, dim3(grid_for(h->np)), dim3(256), 0, h->stream, h->w, h->g, h->m, h->v, h->np, lr, beta1,
                     beta2, eps, c1, c2, h->wb);
  MLPX(hipGetLastError());
  return 0;
}

}  // namespace

extern "C" {

int pdhcg_mlp_create(pdhcg_mlp** out, int32_t n_in, int32_t n_hid, int32_t n_out, int32_t max_batch,
                     void* hip_stream) {
  if (!out) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null handle pointer");
  *out = nullptr;
  if (n_in < 1 || n_hid < 1 || n_out < 1 || max_batch < 1)
    return set_error(PDHCG_ERR_INVALID_ARGUMENT, "network sizes and max_batch must be >= 1");
  pdhcg_mlp* h = new pdhcg_mlp();
  h->n_in = n_in;
  h->n_hid = n_hid;
  h->n_out = n_out;
  h->cap = max_batch;
  h->stream = (hipStream_t)hip_stream;
  const int64_t sizes[6] = {(int64_t)n_in * n_hid, n_hid, (int64_t)n_hid * n_hid, n_hid, (int64_t)n_hid * n_out, n_out};
  int64_t acc = 0;
  for (int k = 0; k < 6; ++k) {
    h->off[k] = acc;
    acc += sizes[k];
  }
  h->np = acc;
  const int64_t B = max_batch;
  bool ok = h->alloc(&h->w, acc) && h->alloc(&h->g, acc) && h->alloc(&h->m, acc) && h->alloc(&h->v, acc) &&
            h->alloc(&h->wb, acc) && h->alloc(&h->xb, B * n_in) && h->alloc(&h->h1, B * n_hid) &&
            h->alloc(&h->h2, B * n_hid) && h->alloc(&h->gob, B * n_out) && h->alloc(&h->d2b, B * n_hid) &&
            h->alloc(&h->d1b, B * n_hid) && h->alloc(&h->out, B * n_out) && h->alloc(&h->go, B * n_out) &&
            h->alloc(&h->d2, B * n_hid) && h->alloc(&h->d1, B * n_hid) && h->alloc(&h->loss, 1) &&
            h->alloc(&h->partial, 2048) && h->alloc(&h->loss_acc, 2) &&
            h->alloc(&h->kpart, (int64_t)kSplitMax * kSplitTiles * GB * GB);
  if (!ok) {
    delete h;
    return set_error(PDHCG_ERR_OUT_OF_MEMORY, "hipMalloc failed for the network");
  }
  if (hipMemsetAsync(h->w, 0, sizeof(float) * acc, h->stream) != hipSuccess ||
      hipMemsetAsync(h->wb, 0, sizeof(uint16_t) * acc, h->stream) != hipSuccess ||
      hipMemsetAsync(h->loss_acc, 0, sizeof(double) * 2, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    delete h;
    return set_error(PDHCG_ERR_HIP, "initialising the network failed");
  }
  *out = h;
  return 0;
}

int64_t pdhcg_mlp_num_params(const pdhcg_mlp* h) { return h ? h->np : 0; }

int pdhcg_mlp_set_params(pdhcg_mlp* h, const float* params) {
  if (!h || !params) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null argument");
  MLPX(hipMemcpyAsync(h->w, params, sizeof(float) * h->np, hipMemcpyHostToDevice, h->stream));
  MLPX(hipMemsetAsync(h->m, 0, sizeof(float) * h->np, h->stream));
  MLPX(hipMemsetAsync(h->v, 0, sizeof(float) * h->np, h->stream));
  hipLaunchKernelGGL(f32_to_bf16, dim3(grid_for(h->np)), dim3(256), 0, h->stream, h->w, h->wb, h->np);
  MLPX(hipGetLastError());
  MLPX(hipStreamSynchronize(h->stream));
  h->t = 0;
  return 0;
}

int pdhcg_mlp_get_params(const pdhcg_mlp* h, float* params) {
  if (!h || !params) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null argument");
  MLPX(hipMemcpyAsync(params, h->w, sizeof(float) * h->np, hipMemcpyDeviceToHost, h->stream));
  MLPX(hipStreamSynchronize(h->stream));
  return 0;
}

int pdhcg_mlp_forward(pdhcg_mlp* h, const float* X, int32_t batch, float* Y) {
  int rc;
  if ((rc = check_batch(h, batch))) return rc;
  if (!X || !Y) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null X or Y");
  if ((rc = run_forward(h, X, nullptr, batch))) return rc;
  MLPX(hipMemcpyAsync(Y, h->out, sizeof(float) * (int64_t)batch * h->n_out, hipMemcpyDeviceToDevice, h->stream));
  MLPX(hipStreamSynchronize(h->stream));
  return 0;
}

int pdhcg_mlp_predict_start(pdhcg_mlp* h, const float* X, int32_t batch, const double* out_mu,
                            const double* out_sd, int32_t n, int32_t n_pair, const int32_t* plus,
                            const int32_t* minus, int32_t n_rest, const int32_t* rest, int32_t m, double* x0,
                            double* y0) {
  if (!h) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null network handle");
  if (batch < 1) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "batch must be >= 1");
  if (!X || !out_mu || !out_sd || !x0 || (m > 0 && !y0))
    return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null input or output array");
  if (n < 0 || n_pair < 0 || n_rest < 0 || m < 0 || n + n_pair + n_rest != h->n_out || 2 * n_pair + n_rest != m)
    return set_error(PDHCG_ERR_INVALID_ARGUMENT,
                     "need n + n_pair + n_rest = n_out and 2 n_pair + n_rest = m (every row of y once)");
  if ((n_pair > 0 && (!plus || !minus)) || (n_rest > 0 && !rest))
    return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null row index array");
  int rc;
  for (int64_t r0 = 0; r0 < batch; r0 += h->cap) {  // chunks of the workspace's rows
    const int rows = (int)std::min<int64_t>(h->cap, batch - r0);
    if ((rc = run_forward(h, X + r0 * h->n_in, nullptr, rows))) return rc;
    const int64_t total = (int64_t)rows * h->n_out;
    hipLaunchKernelGGL(decode_start, dim3(grid_for(total)), dim3(256), 0, h->stream, h->out, rows, h->n_out, out_mu,
                       out_sd, n, n_pair, plus, minus, rest, m, r0, x0, y0);
    MLPX(hipGetLastError());
  }
  MLPX(hipStreamSynchronize(h->stream));
  return 0;
}

int pdhcg_mlp_loss_grad(pdhcg_mlp* h, const float* X, const float* T, int32_t batch, float* loss, float* grads) {
  int rc;
  if ((rc = check_batch(h, batch))) return rc;
  if (!X || !T) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null X or T");
  if ((rc = queue_loss_grad(h, X, T, nullptr, batch))) return rc;
  if (loss) MLPX(hipMemcpyAsync(loss, h->loss, sizeof(float), hipMemcpyDeviceToHost, h->stream));
  if (grads) MLPX(hipMemcpyAsync(grads, h->g, sizeof(float) * h->np, hipMemcpyDeviceToHost, h->stream));
  MLPX(hipStreamSynchronize(h->stream));
  return 0;
}

int pdhcg_mlp_train_step(pdhcg_mlp* h, const float* X, const float* T, const int32_t* rows, int32_t batch, float lr,
                         float beta1, float beta2, float eps) {
  int rc;
  if ((rc = check_batch(h, batch))) return rc;
  if (!X || !T) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null X or T");
  if ((rc = queue_loss_grad(h, X, T, rows, batch))) return rc;
  return queue_adam(h, lr, beta1, beta2, eps);
}

int pdhcg_mlp_take_loss(pdhcg_mlp* h, double* sum, int64_t* steps) {
  if (!h) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null network handle");
  double acc[2] = {0.0, 0.0};
  MLPX(hipMemcpyAsync(acc, h->loss_acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
  MLPX(hipMemsetAsync(h->loss_acc, 0, sizeof(double) * 2, h->stream));
  MLPX(hipStreamSynchronize(h->stream));
  if (sum) *sum = acc[0];
  if (steps) *steps = (int64_t)acc[1];
  return 0;
}

int pdhcg_mlp_adam_step(pdhcg_mlp* h, float lr, float beta1, float beta2, float eps) {
  if (!h) return set_error(PDHCG_ERR_INVALID_ARGUMENT, "null network handle");
  int rc;
  if ((rc = queue_adam(h, lr, beta1, beta2, eps))) return rc;
  MLPX(hipStreamSynchronize(h->stream));
  return 0;
}

void pdhcg_mlp_destroy(pdhcg_mlp* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

}  // extern "C"
