// mlp.hip -- the triage network's kernels (fp32): 128 -> 256 -> 256 -> 1 with
// ReLU, mean binary cross-entropy on logits, Adam.  Parameters are one flat
// vector: W1[256x128], b1[256], W2[256x256], b2[256], w3[256], b3[1].
//
// All matrix products go through one tiled GEMM (64x64 tiles, 16-deep K
// steps staged in LDS, 4x4 outputs per thread) whose operands are read
// through strides, so transposed operands need no copies, and whose epilogue
// fuses the bias, the ReLU of an operand and the ReLU derivative mask.
// Long reductions (the weight gradients sum over the minibatch) are split
// over K into slices of at most 256 that run as separate workgroups and are
// added in slice order afterwards: more parallelism for the 256x256
// outputs, and shorter fp32 accumulation chains.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.h"

namespace rc {

constexpr int TM = 64, TN = 64, TK = 16;

struct GemmArgs {
  const float* A;        // A(m, k) = A[row_a(m) * sam + k * sak]
  const float* B;        // B(k, n) = B[row_b(k) * sbk + n * sbn]
  const uint32_t* rows_a;  // row_a(m) = rows_a ? rows_a[m] : m
  const uint32_t* rows_b;  // row_b(k) = rows_b ? rows_b[k] : k
  float* C;              // C(m, n) = C[m * ldc + n]
  const float* bias;     // per column n (nullptr: none)
  const float* mask;     // C(m, n) *= (mask[m * ldc + n] > 0) (nullptr: none)
  long long sam, sak, sbk, sbn, ldc;
  int M, N, K;
  int relu_a, relu_b;    // read relu(A) / relu(B)
  float* partial;        // split K: slice z writes raw sums to partial[(z * M + m) * N + n]
  int kchunk;            // K range of one slice (a multiple of TK)
};

__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  __shared__ float As[TK][TM + 1];
  __shared__ float Bs[TK][TN + 1];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = blockIdx.z * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  float acc[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  for (int k0 = kb; k0 < ke; k0 += TK) {
    for (int r = 0; r < 4; ++r) {
      const int e = t + r * 256;
      {  // A tile: 64 rows x 16 k
        const int row = e / TK, kk = e % TK;
        const int m = m0 + row, k = k0 + kk;
        float v = 0.f;
        if (m < g.M && k < ke) {
          const long long r = g.rows_a ? (long long)g.rows_a[m] : (long long)m;
          v = g.A[r * g.sam + (long long)k * g.sak];
          if (g.relu_a) v = v > 0.f ? v : 0.f;
        }
        As[kk][row] = v;
      }
      {  // B tile: 16 k x 64 columns
        const int kk = e / TN, col = e % TN;
        const int k = k0 + kk, n = n0 + col;
        float v = 0.f;
        if (k < ke && n < g.N) {
          const long long r = g.rows_b ? (long long)g.rows_b[k] : (long long)k;
          v = g.B[r * g.sbk + (long long)n * g.sbn];
          if (g.relu_b) v = v > 0.f ? v : 0.f;
        }
        Bs[kk][col] = v;
      }
    }
    __syncthreads();
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], b[4];
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= g.M) continue;
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n >= g.N) continue;
      float v = acc[i][j];
      if (g.partial) {
        g.partial[((long long)blockIdx.z * g.M + m) * g.N + n] = v;
        continue;
      }
      if (g.bias) v += g.bias[n];
      if (g.mask && !(g.mask[(long long)m * g.ldc + n] > 0.f)) v = 0.f;
      g.C[(long long)m * g.ldc + n] = v;
    }
  }
}

// C = sum of the K slices in slice order, then the epilogue
__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmArgs g, int slices) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)g.M * g.N) return;
  const int m = (int)(e / g.N), n = (int)(e % g.N);
  float v = 0.f;
  for (int z = 0; z < slices; ++z) v += g.partial[(long long)z * g.M * g.N + e];
  if (g.bias) v += g.bias[n];
  if (g.mask && !(g.mask[(long long)m * g.ldc + n] > 0.f)) v = 0.f;
  g.C[(long long)m * g.ldc + n] = v;
}

constexpr int SPLIT_K = 256, MAX_SLICES = 64;

// `partial` holds MAX_SLICES * M * N floats (used when K > SPLIT_K)
static hipError_t gemm(GemmArgs g, float* partial, hipStream_t st) {
  int slices = 1;
  g.kchunk = g.K;
  g.partial = nullptr;
  if (g.K > SPLIT_K && partial) {
    int chunk = SPLIT_K;
    if ((g.K + chunk - 1) / chunk > MAX_SLICES) chunk = (((g.K + MAX_SLICES - 1) / MAX_SLICES) + TK - 1) / TK * TK;
    g.kchunk = chunk;
    slices = (g.K + chunk - 1) / chunk;
    g.partial = partial;
  }
  dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, slices);
  hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, st, g);
  if (slices > 1) {
    const long long total = (long long)g.M * g.N;
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g, slices);
  }
  return hipGetLastError();
}

// z[i] = relu(A2[i]) . w3 + b3 : one wave per row
__global__ __launch_bounds__(256) void head_kernel(const float* A2, const float* w3, const float* b3, float* z, int n) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  float s = 0.f;
  for (int j = lane; j < MLP_H; j += 64) {
    const float h = A2[(long long)row * MLP_H + j];
    s = fmaf(h > 0.f ? h : 0.f, w3[j], s);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if (lane == 0) z[row] = s + b3[0];
}

// dz = (sigmoid(z) - y) / n; z is overwritten with the row's loss term
// (softplus(z) - y z) / n, summed afterwards in a fixed order
__global__ __launch_bounds__(256) void bce_kernel(float* z, const float* y, const uint32_t* rows, float* dz, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float zi = z[i], yi = y[rows ? rows[i] : (uint32_t)i];
  const float sig = 1.f / (1.f + expf(-zi));
  dz[i] = (sig - yi) / (float)n;
  const float sp = zi > 0.f ? zi + log1pf(expf(-zi)) : log1pf(expf(zi));
  z[i] = (sp - yi * zi) / (float)n;
}

// dA2[i][j] = dz[i] * w3[j] * (A2[i][j] > 0)
__global__ __launch_bounds__(256) void head_back_kernel(const float* dz, const float* w3, const float* A2, float* dA2,
                                                        long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long i = e / MLP_H;
  const int j = (int)(e % MLP_H);
  dA2[e] = A2[e] > 0.f ? dz[i] * w3[j] : 0.f;
}

// Column sums out[j] = sum_i f(M[i][j]) * (w ? w[i] : 1), f = relu if relu_m,
// in two deterministic stages: blocks of 64 columns x one row split write
// partial sums, then one thread per column adds the splits in order.
constexpr int CS_SPLITS = 64;

__global__ __launch_bounds__(256) void colsum_partial_kernel(const float* Mx, const float* w, float* partial, int n,
                                                             int cols, int relu_m, int rows_per_split) {
  __shared__ float part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int r0 = blockIdx.y * rows_per_split;
  const int r1 = min(n, r0 + rows_per_split);
  float s = 0.f;
  if (j < cols) {
    for (int i = r0 + wave; i < r1; i += 4) {
      float v = Mx[(long long)i * cols + j];
      if (relu_m) v = v > 0.f ? v : 0.f;
      s = fmaf(v, w ? w[i] : 1.f, s);
    }
  }
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && j < cols)
    partial[(long long)blockIdx.y * cols + j] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

__global__ __launch_bounds__(256) void colsum_final_kernel(const float* partial, int splits, int cols, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int k = 0; k < splits; ++k) s += partial[(long long)k * cols + j];
  out[j] = s;
}

static hipError_t colsum(const float* Mx, const float* w, float* out, int n, int cols, int relu_m, float* partial,
                         hipStream_t st) {
  const int rows = n > 0 ? (n + CS_SPLITS - 1) / CS_SPLITS : 1;
  const int splits = n > 0 ? (n + rows - 1) / rows : 1;
  hipLaunchKernelGGL(colsum_partial_kernel, dim3((cols + 63) / 64, splits), dim3(256), 0, st, Mx, w, partial, n, cols,
                     relu_m, rows);
  hipLaunchKernelGGL(colsum_final_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, (const float*)partial, splits,
                     cols, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void sum_kernel(const float* v, int n, float* out) {
  __shared__ float part[4];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = part[0] + part[1] + part[2] + part[3];
}

// Adam (Kingma and Ba): m, v moments, bias-corrected, step counts from 1
__global__ __launch_bounds__(256) void adam_kernel(float* theta, float* m, float* v, const float* g, int n, float lr,
                                                   float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = MLP_B1 * m[i] + (1.f - MLP_B1) * gi;
  const float vi = MLP_B2 * v[i] + (1.f - MLP_B2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mhat = mi / c1, vhat = vi / c2;
  theta[i] -= lr * mhat / (sqrtf(vhat) + MLP_EPS);
}

// ---------------------------------------------------------------------------
size_t mlp_ws_bytes(uint32_t n) {
  // A1, A2, dA2, dA1 [n x 256]; z, dz [n]; gradient [params]; column-sum
  // partials; split-K partials of a 256 x 256 product
  return (size_t)n * MLP_H * 4 * 4 + (size_t)n * 4 * 2 + (size_t)MLP_PARAMS * 4 + (size_t)CS_SPLITS * MLP_H * 4 +
         (size_t)MAX_SLICES * MLP_H * MLP_H * 4;
}

static const float* P_W1(const float* p) { return p; }
static const float* P_b1(const float* p) { return p + MLP_H * MLP_IN; }
static const float* P_W2(const float* p) { return p + MLP_H * MLP_IN + MLP_H; }
static const float* P_b2(const float* p) { return p + MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H; }
static const float* P_w3(const float* p) { return p + MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H; }
static const float* P_b3(const float* p) { return p + MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + 2 * MLP_H; }

struct MlpWs {
  float *A1, *A2, *dA2, *dA1, *z, *dz, *grad, *partial, *kpart;
};
static MlpWs carve(void* ws, uint32_t n) {
  float* f = (float*)ws;
  MlpWs w;
  w.A1 = f; f += (size_t)n * MLP_H;
  w.A2 = f; f += (size_t)n * MLP_H;
  w.dA2 = f; f += (size_t)n * MLP_H;
  w.dA1 = f; f += (size_t)n * MLP_H;
  w.z = f; f += n;
  w.dz = f; f += n;
  w.grad = f; f += MLP_PARAMS;
  w.partial = f; f += (size_t)CS_SPLITS * MLP_H;
  w.kpart = f;
  return w;
}

static hipError_t forward_into(const float* theta, const float* X, const uint32_t* rows, uint32_t n, const MlpWs& w,
                               float* logits, hipStream_t st) {
  GemmArgs g{};
  // A1 = X[rows] W1^T + b1
  g.A = X; g.sam = MLP_IN; g.sak = 1; g.rows_a = rows;
  g.B = P_W1(theta); g.sbk = 1; g.sbn = MLP_IN;
  g.C = w.A1; g.ldc = MLP_H; g.bias = P_b1(theta);
  g.M = (int)n; g.N = MLP_H; g.K = MLP_IN;
  hipError_t e = gemm(g, w.kpart, st);
  if (e != hipSuccess) return e;
  // A2 = relu(A1) W2^T + b2
  g = GemmArgs{};
  g.A = w.A1; g.sam = MLP_H; g.sak = 1; g.relu_a = 1;
  g.B = P_W2(theta); g.sbk = 1; g.sbn = MLP_H;
  g.C = w.A2; g.ldc = MLP_H; g.bias = P_b2(theta);
  g.M = (int)n; g.N = MLP_H; g.K = MLP_H;
  e = gemm(g, w.kpart, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(head_kernel, dim3((n + 3) / 4), dim3(256), 0, st, (const float*)w.A2, P_w3(theta), P_b3(theta),
                     logits, (int)n);
  return hipGetLastError();
}

hipError_t mlp_forward(const float* theta, const float* X, uint32_t n, float* logits, void* ws, hipStream_t st) {
  return forward_into(theta, X, nullptr, n, carve(ws, n), logits, st);
}

hipError_t mlp_grad(const float* theta, const float* X, const float* y, const uint32_t* rows, uint32_t n,
                    float* grad, float* loss, void* ws, hipStream_t st) {
  MlpWs w = carve(ws, n);
  hipError_t e = forward_into(theta, X, rows, n, w, w.z, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bce_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w.z, y, rows, w.dz, (int)n);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, (const float*)w.z, (int)n, loss);
  float* gW1 = grad;
  float* gb1 = grad + MLP_H * MLP_IN;
  float* gW2 = gb1 + MLP_H;
  float* gb2 = gW2 + MLP_H * MLP_H;
  float* gw3 = gb2 + MLP_H;
  float* gb3 = gw3 + MLP_H;
  // head: gw3 = relu(A2)^T dz, gb3 = sum dz, dA2 = dz w3 * (A2 > 0)
  if ((e = colsum(w.A2, w.dz, gw3, (int)n, MLP_H, 1, w.partial, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, (const float*)w.dz, (int)n, gb3);
  const long long tot = (long long)n * MLP_H;
  hipLaunchKernelGGL(head_back_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, (const float*)w.dz,
                     P_w3(theta), (const float*)w.A2, w.dA2, tot);
  // gW2 = dA2^T relu(A1); gb2 = column sums of dA2
  GemmArgs g{};
  g.A = w.dA2; g.sam = 1; g.sak = MLP_H;
  g.B = w.A1; g.sbk = MLP_H; g.sbn = 1; g.relu_b = 1;
  g.C = gW2; g.ldc = MLP_H;
  g.M = MLP_H; g.N = MLP_H; g.K = (int)n;
  if ((e = gemm(g, w.kpart, st)) != hipSuccess) return e;
  if ((e = colsum(w.dA2, nullptr, gb2, (int)n, MLP_H, 0, w.partial, st)) != hipSuccess) return e;
  // dA1 = (dA2 W2) * (A1 > 0)
  g = GemmArgs{};
  g.A = w.dA2; g.sam = MLP_H; g.sak = 1;
  g.B = P_W2(theta); g.sbk = MLP_H; g.sbn = 1;
  g.C = w.dA1; g.ldc = MLP_H; g.mask = w.A1;
  g.M = (int)n; g.N = MLP_H; g.K = MLP_H;
  if ((e = gemm(g, w.kpart, st)) != hipSuccess) return e;
  // gW1 = dA1^T X[rows]; gb1 = column sums of dA1
  g = GemmArgs{};
  g.A = w.dA1; g.sam = 1; g.sak = MLP_H;
  g.B = X; g.sbk = MLP_IN; g.sbn = 1; g.rows_b = rows;
  g.C = gW1; g.ldc = MLP_IN;
  g.M = MLP_H; g.N = MLP_IN; g.K = (int)n;
  if ((e = gemm(g, w.kpart, st)) != hipSuccess) return e;
  if ((e = colsum(w.dA1, nullptr, gb1, (int)n, MLP_H, 0, w.partial, st)) != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t mlp_train_step(float* theta, float* m, float* v, uint32_t step, const float* X, const float* y,
                          const uint32_t* rows, uint32_t n, float lr, float* loss, void* ws, hipStream_t st) {
  MlpWs w = carve(ws, n);
  hipError_t e = mlp_grad(theta, X, y, rows, n, w.grad, loss, ws, st);
  if (e != hipSuccess) return e;
  const float c1 = 1.f - powf(MLP_B1, (float)step), c2 = 1.f - powf(MLP_B2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, st, theta, m, v,
                     (const float*)w.grad, (int)MLP_PARAMS, lr, c1, c2);
  return hipGetLastError();
}

}  // namespace rc
