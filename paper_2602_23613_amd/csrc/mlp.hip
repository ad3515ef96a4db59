// Learned-setup surrogate network (gfx950): a 64 -> 128 -> 128 -> 64 MLP that
// maps a normalised extension block D^{-1/2} A_BB D^{-1/2} (size <= 8) to its
// inverse, trained on the exact local solves of the harmonic extension
// (eq. (sparseP)).  Matrix products use MFMA (v_mfma_f32_16x16x32_bf16, BF16
// operands, FP32 accumulation); master weights and Adam state are FP32.  At
// inference the prediction is refined in FP64 by Newton-Schulz steps and
// accepted only if ||Ahat W - I||_F <= tol; otherwise the exact solve is used.
#include "mlp.hpp"

#include <hip/hip_runtime.h>

namespace hamg {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even (finite inputs)
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

static unsigned grid1(int64_t n, int bs = 256) {
  int64_t g = (n + bs - 1) / bs;
  if (g > 65535 * 8) g = 65535 * 8;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// C[M x N] (+)= sum_k A(m, k) B(k, n), BF16 operands with arbitrary strides,
// FP32 accumulation.  One wavefront per 16 x 16 tile of C; M, N, K multiples
// of 16.  K goes in steps of 32 through gfx950's v_mfma_f32_16x16x32_bf16
// (lane l holds A(l % 16, 8 (l / 16) + t) and B(8 (l / 16) + t, l % 16),
// t = 0..7), a last step of 16 through v_mfma_f32_16x16x16_bf16 (lane l
// holds A(l % 16, 4 (l / 16) + t) and B(4 (l / 16) + t, l % 16), t = 0..3);
// both leave C(4 (l / 16) + t, l % 16) in lane l, t = 0..3.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t* __restrict__ A,
                                                   int64_t lda_m, int64_t lda_k,
                                                   const uint16_t* __restrict__ B, int64_t ldb_k,
                                                   int64_t ldb_n, float* __restrict__ C, int64_t ldc,
                                                   int accumulate) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int tiles_n = N / 16;
  const int64_t tile = (int64_t)blockIdx.x * (blockDim.x / 64) + wave;
  const int64_t tm = tile / tiles_n, tn = tile % tiles_n;
  if (tm * 16 >= M) return;   // whole wavefront leaves together
  const int i = lane % 16, kq = 4 * (lane / 16), kq8 = 8 * (lane / 16);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const uint16_t* Ap = A + (tm * 16 + i) * lda_m;
  const uint16_t* Bp = B + (tn * 16 + i) * ldb_n;
  int k0 = 0;
  for (; k0 + 32 <= K; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      a[t] = __builtin_bit_cast(__bf16, Ap[(int64_t)(k0 + kq8 + t) * lda_k]);
      b[t] = __builtin_bit_cast(__bf16, Bp[(int64_t)(k0 + kq8 + t) * ldb_k]);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  if (k0 < K) {   // K = 16 (mod 32)
    bf16x4 a, b;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a[t] = (short)Ap[(int64_t)(k0 + kq + t) * lda_k];
      b[t] = (short)Bp[(int64_t)(k0 + kq + t) * ldb_k];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float* c = C + (tm * 16 + kq + t) * ldc + tn * 16 + i;
    *c = accumulate ? *c + acc[t] : acc[t];
  }
}

void gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t lda_m, int64_t lda_k,
               const uint16_t* B, int64_t ldb_k, int64_t ldb_n, float* C, int64_t ldc, int accumulate,
               hipStream_t st) {
  int64_t tiles = (int64_t)(M / 16) * (N / 16);
  unsigned grid = (unsigned)((tiles + 3) / 4);
  hipLaunchKernelGGL(k_gemm_bf16, dim3(grid), dim3(256), 0, st, M, N, K, A, lda_m, lda_k, B, ldb_k,
                     ldb_n, C, ldc, accumulate);
}

// ---------------------------------------------------------------------------
// elementwise pieces
// ---------------------------------------------------------------------------
// Z += bias (row-broadcast); H = relu(Z) as BF16
__global__ void k_bias_relu_bf16(int64_t rows, int cols, float* __restrict__ Z,
                                 const float* __restrict__ bias, uint16_t* __restrict__ H) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < rows * cols;
       t += (int64_t)gridDim.x * blockDim.x) {
    float z = Z[t] + bias[t % cols];
    Z[t] = z;
    H[t] = to_bf16(z > 0.f ? z : 0.f);
  }
}
// Y += bias
__global__ void k_bias(int64_t rows, int cols, float* __restrict__ Y, const float* __restrict__ bias) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < rows * cols;
       t += (int64_t)gridDim.x * blockDim.x)
    Y[t] += bias[t % cols];
}
// G = G * (Z > 0); Gb = bf16(G)
__global__ void k_relu_mask_bf16(int64_t n, float* __restrict__ G, const float* __restrict__ Z,
                                 uint16_t* __restrict__ Gb) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    float g = Z[t] > 0.f ? G[t] : 0.f;
    G[t] = g;
    Gb[t] = to_bf16(g);
  }
}
__global__ void k_to_bf16(int64_t n, const float* __restrict__ a, uint16_t* __restrict__ b) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    b[t] = to_bf16(a[t]);
}
// column sums (bias gradients), fixed order
__global__ void k_colsum(int64_t rows, int cols, const float* __restrict__ G, float* __restrict__ out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int64_t r = 0; r < rows; ++r) s += G[r * cols + c];
  out[c] = s;
}
// Training loss of one sample: the error of the predicted inverse against
// the exact one in the metric of the block, L = ||Ahat (W - W*)||_F^2, which
// equals the refinement residual ||Ahat W - I||_F^2 that decides acceptance
// (Ahat W* = I).  W, W* and Ahat are symmetric 8 x 8 matrices stored as packed
// lower triangles (36 of the 64 outputs).  dL/dE = 2 Ahat^2 E =: G with
// E = W - W*; a packed off-diagonal entry feeds E_ij and E_ji, so its gradient
// is G_ij + G_ji.  Rows r >= nvalid (batch padding) get zero gradient; the
// loss is averaged over the nvalid rows.  ahat_idx (may be NULL) maps batch
// rows to rows of Ahat.
__global__ void k_aloss(int64_t rows, const float* __restrict__ Y, const float* __restrict__ T,
                        const double* __restrict__ Ahat, const int32_t* __restrict__ ahat_idx,
                        int64_t nvalid, float inv_n, float* __restrict__ dY,
                        float* __restrict__ row_loss) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float* g = dY + r * MLP_OUT;
  if (r >= nvalid) {
    for (int q = 0; q < MLP_OUT; ++q) g[q] = 0.f;
    row_loss[r] = 0.f;
    return;
  }
  const int64_t a = ahat_idx ? (int64_t)ahat_idx[r] : r;
  const double* ap = Ahat + a * 36;
  double A[8][8], E[8][8], AE[8][8];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j <= i; ++j) {
      const int q = i * (i + 1) / 2 + j;
      A[i][j] = A[j][i] = ap[q];
      E[i][j] = E[j][i] = (double)Y[r * MLP_OUT + q] - (double)T[r * MLP_OUT + q];
    }
  double loss = 0.0;
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) {
      double v = 0.0;
      for (int k = 0; k < 8; ++k) v += A[i][k] * E[k][j];
      AE[i][j] = v;
      loss += v * v;
    }
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j <= i; ++j) {
      double gij = 0.0, gji = 0.0;   // (Ahat AE)_ij and (Ahat AE)_ji
      for (int k = 0; k < 8; ++k) {
        gij += A[i][k] * AE[k][j];
        gji += A[j][k] * AE[k][i];
      }
      const double d = (i == j) ? 2.0 * gij : 2.0 * (gij + gji);
      g[i * (i + 1) / 2 + j] = (float)(d * inv_n);
    }
  for (int q = 36; q < MLP_OUT; ++q) g[q] = 0.f;
  row_loss[r] = (float)loss;
}
// Adam on the FP32 master parameters (bias-corrected), refresh BF16 copies
__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    float gi = g[t];
    float mi = b1 * m[t] + (1.f - b1) * gi;
    float vi = b2 * v[t] + (1.f - b2) * gi * gi;
    m[t] = mi;
    v[t] = vi;
    p[t] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}
// gather rows idx[0..n) of X (bf16, 64 wide) and T (fp32, 64 wide); pad rows get zeros
__global__ void k_gather_rows(int64_t n, int64_t npad, const int32_t* __restrict__ idx,
                              const uint16_t* __restrict__ X, const float* __restrict__ T,
                              uint16_t* __restrict__ Xb, float* __restrict__ Tb) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad * 64;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = t / 64, c = t % 64;
    if (r < n) {
      Xb[t] = X[(int64_t)idx[r] * 64 + c];
      if (Tb) Tb[t] = T[(int64_t)idx[r] * 64 + c];
    } else {
      Xb[t] = 0;
      if (Tb) Tb[t] = 0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// block features, exact targets (one thread per extension block, size <= 8)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }

__global__ void k_block_features(int64_t nb, const int64_t* __restrict__ bptr,
                                 const int32_t* __restrict__ bdofs, const int64_t* __restrict__ Aptr,
                                 const int32_t* __restrict__ Acol, const double* __restrict__ Aval,
                                 double eligible_max, uint16_t* __restrict__ X, float* __restrict__ T,
                                 double* __restrict__ Ahat, double* __restrict__ dsq,
                                 int8_t* __restrict__ eligible) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t d0 = bptr[b];
  const int s = (int)(bptr[b + 1] - d0);
  uint16_t* x = X + b * MLP_IN;
  float* t = T + b * MLP_OUT;
  double* ah = Ahat + b * 36;
  double* dq = dsq + b * 8;
  for (int q = 0; q < MLP_IN; ++q) x[q] = 0;
  for (int q = 0; q < MLP_OUT; ++q) t[q] = 0.f;
  if (s > MLP_SMAX) {
    eligible[b] = 0;
    return;
  }
  double M[36];   // packed lower triangle of the 8 x 8 normalised block (identity padded)
  double dg[8];
  for (int i = 0; i < 8; ++i) dg[i] = 1.0;
  for (int i = 0; i < s; ++i) {
    const int32_t e = bdofs[d0 + i];
    const int64_t q0 = Aptr[e];
    const int len = (int)(Aptr[e + 1] - q0);
    for (int j = 0; j <= i; ++j) {
      const int32_t d = bdofs[d0 + j];
      int lo = 0, hi = len;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (Acol[q0 + mid] < d) lo = mid + 1; else hi = mid;
      }
      M[pk(i, j)] = (lo < len && Acol[q0 + lo] == d) ? Aval[q0 + lo] : 0.0;
    }
    dg[i] = M[pk(i, i)];
  }
  bool ok = true;
  for (int i = 0; i < s; ++i) ok = ok && dg[i] > 0.0;
  for (int i = 0; i < 8; ++i) dq[i] = ok ? sqrt(dg[i]) : 1.0;
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j <= i; ++j) {
      double v;
      if (i < s && j < s) v = ok ? M[pk(i, j)] / (dq[i] * dq[j]) : 0.0;
      else v = (i == j) ? 1.0 : 0.0;
      M[pk(i, j)] = v;
      ah[pk(i, j)] = v;
    }
  // Cholesky of the normalised block and its inverse (exact target)
  double L[36];
  for (int q = 0; q < 36; ++q) L[q] = M[q];
  for (int j = 0; j < 8 && ok; ++j) {
    double a = L[pk(j, j)];
    for (int k = 0; k < j; ++k) a -= L[pk(j, k)] * L[pk(j, k)];
    if (!(a > 0.0)) { ok = false; break; }
    const double dj = sqrt(a);
    L[pk(j, j)] = dj;
    for (int i = j + 1; i < 8; ++i) {
      double v = L[pk(i, j)];
      for (int k = 0; k < j; ++k) v -= L[pk(i, k)] * L[pk(j, k)];
      L[pk(i, j)] = v / dj;
    }
  }
  double W[36];
  double wmax = 0.0;
  if (ok) {
    for (int c = 0; c < 8; ++c) {   // column c of the inverse
      double y[8];
      for (int i = 0; i < 8; ++i) {
        double v = (i == c) ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) v -= L[pk(i, k)] * y[k];
        y[i] = v / L[pk(i, i)];
      }
      for (int i = 7; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < 8; ++k) v -= L[pk(k, i)] * y[k];
        y[i] = v / L[pk(i, i)];
      }
      for (int i = c; i < 8; ++i) W[pk(i, c)] = y[i];
    }
    for (int q = 0; q < 36; ++q) wmax = fmax(wmax, fabs(W[q]));
  }
  eligible[b] = (ok && wmax <= eligible_max) ? 1 : 0;
  // features: packed normalised block, then centred log10 diagonal
  double lsum = 0.0;
  for (int i = 0; i < s; ++i) lsum += ok ? log10(dg[i]) : 0.0;
  for (int q = 0; q < 36; ++q) x[q] = to_bf16((float)M[q]);
  for (int i = 0; i < s; ++i) x[36 + i] = to_bf16((float)(ok ? log10(dg[i]) - lsum / s : 0.0));
  for (int q = 0; q < 36; ++q) t[q] = ok ? (float)W[q] : 0.f;
}

// ---------------------------------------------------------------------------
// inference: Newton-Schulz refinement of the predicted inverse and the check
// ---------------------------------------------------------------------------
__global__ void k_refine_check(int64_t nb, const int64_t* __restrict__ bptr,
                               const int8_t* __restrict__ eligible, const float* __restrict__ Y,
                               const double* __restrict__ Ahat, int steps, double tol,
                               double* __restrict__ Wout, int8_t* __restrict__ accepted,
                               float* __restrict__ resid) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  accepted[b] = 0;
  resid[b] = -1.f;
  if (!eligible[b]) return;
  const int s = (int)(bptr[b + 1] - bptr[b]);
  double A[64], W[64], R[64];
  const double* ah = Ahat + b * 36;
  const float* y = Y + b * MLP_OUT;
  for (int i = 0; i < s; ++i)
    for (int j = 0; j <= i; ++j) {
      A[i * 8 + j] = A[j * 8 + i] = ah[pk(i, j)];
      W[i * 8 + j] = W[j * 8 + i] = (double)y[pk(i, j)];
    }
  double r2 = 0.0;
  for (int it = 0; it <= steps; ++it) {
    // R = A W - I
    r2 = 0.0;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        double v = (i == j) ? -1.0 : 0.0;
        for (int k = 0; k < s; ++k) v += A[i * 8 + k] * W[k * 8 + j];
        R[i * 8 + j] = v;
        r2 += v * v;
      }
    if (it == steps || !(r2 < 1.0)) break;
    // W <- W (2I - A W) = W - W R
    double Wn[64];
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        double v = W[i * 8 + j];
        for (int k = 0; k < s; ++k) v -= W[i * 8 + k] * R[k * 8 + j];
        Wn[i * 8 + j] = v;
      }
    for (int i = 0; i < s; ++i)   // keep it symmetric
      for (int j = 0; j <= i; ++j) W[i * 8 + j] = W[j * 8 + i] = 0.5 * (Wn[i * 8 + j] + Wn[j * 8 + i]);
  }
  const double r = sqrt(r2);
  resid[b] = (float)r;
  if (r <= tol) {
    accepted[b] = 1;
    double* w = Wout + b * 36;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j <= i; ++j) w[pk(i, j)] = W[i * 8 + j];
  }
}

// ---------------------------------------------------------------------------
// host-side network driver
// ---------------------------------------------------------------------------
void mlp_forward(const MlpDev& m, const uint16_t* X, int64_t n, MlpWork& w, float* Y, hipStream_t st) {
  // Z1 = X W1 + b1, H1 = relu
  gemm_bf16((int)n, MLP_HID, MLP_IN, X, MLP_IN, 1, m.Wb1, MLP_HID, 1, w.Z1, MLP_HID, 0, st);
  hipLaunchKernelGGL(k_bias_relu_bf16, dim3(grid1(n * MLP_HID)), dim3(256), 0, st, n, MLP_HID, w.Z1,
                     m.b1, w.H1);
  gemm_bf16((int)n, MLP_HID, MLP_HID, w.H1, MLP_HID, 1, m.Wb2, MLP_HID, 1, w.Z2, MLP_HID, 0, st);
  hipLaunchKernelGGL(k_bias_relu_bf16, dim3(grid1(n * MLP_HID)), dim3(256), 0, st, n, MLP_HID, w.Z2,
                     m.b2, w.H2);
  gemm_bf16((int)n, MLP_OUT, MLP_HID, w.H2, MLP_HID, 1, m.Wb3, MLP_OUT, 1, Y, MLP_OUT, 0, st);
  hipLaunchKernelGGL(k_bias, dim3(grid1(n * MLP_OUT)), dim3(256), 0, st, n, MLP_OUT, Y, m.b3);
}

void mlp_backward(const MlpDev& m, const uint16_t* X, int64_t n, MlpWork& w, const float* dY,
                  float* grad, hipStream_t st) {
  float* gW1 = grad + MLP_OFF_W1;
  float* gb1 = grad + MLP_OFF_B1;
  float* gW2 = grad + MLP_OFF_W2;
  float* gb2 = grad + MLP_OFF_B2;
  float* gW3 = grad + MLP_OFF_W3;
  float* gb3 = grad + MLP_OFF_B3;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(n * MLP_OUT)), dim3(256), 0, st, n * MLP_OUT, dY, w.dYb);
  // gW3 = H2^T dYb ; gb3 = colsum dY
  gemm_bf16(MLP_HID, MLP_OUT, (int)n, w.H2, 1, MLP_HID, w.dYb, MLP_OUT, 1, gW3, MLP_OUT, 0, st);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(MLP_OUT), 0, st, n, MLP_OUT, dY, gb3);
  // dH2 = (dYb W3^T) * (Z2 > 0)
  gemm_bf16((int)n, MLP_HID, MLP_OUT, w.dYb, MLP_OUT, 1, m.Wb3, 1, MLP_OUT, w.dH, MLP_HID, 0, st);
  hipLaunchKernelGGL(k_relu_mask_bf16, dim3(grid1(n * MLP_HID)), dim3(256), 0, st, n * MLP_HID, w.dH,
                     w.Z2, w.dHb);
  gemm_bf16(MLP_HID, MLP_HID, (int)n, w.H1, 1, MLP_HID, w.dHb, MLP_HID, 1, gW2, MLP_HID, 0, st);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(MLP_HID), 0, st, n, MLP_HID, w.dH, gb2);
  // dH1 = (dH2b W2^T) * (Z1 > 0)
  gemm_bf16((int)n, MLP_HID, MLP_HID, w.dHb, MLP_HID, 1, m.Wb2, 1, MLP_HID, w.dH, MLP_HID, 0, st);
  hipLaunchKernelGGL(k_relu_mask_bf16, dim3(grid1(n * MLP_HID)), dim3(256), 0, st, n * MLP_HID, w.dH,
                     w.Z1, w.dHb);
  gemm_bf16(MLP_IN, MLP_HID, (int)n, X, 1, MLP_IN, w.dHb, MLP_HID, 1, gW1, MLP_HID, 0, st);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(MLP_HID), 0, st, n, MLP_HID, w.dH, gb1);
}

void mlp_refresh_bf16(MlpDev& m, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(MLP_IN * MLP_HID)), dim3(256), 0, st,
                     (int64_t)MLP_IN * MLP_HID, m.master + MLP_OFF_W1, m.Wb1);
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(MLP_HID * MLP_HID)), dim3(256), 0, st,
                     (int64_t)MLP_HID * MLP_HID, m.master + MLP_OFF_W2, m.Wb2);
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(MLP_HID * MLP_OUT)), dim3(256), 0, st,
                     (int64_t)MLP_HID * MLP_OUT, m.master + MLP_OFF_W3, m.Wb3);
}

void mlp_adam(MlpDev& m, float lr, hipStream_t st) {
  m.step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float c1 = 1.f - powf(b1, (float)m.step), c2 = 1.f - powf(b2, (float)m.step);
  hipLaunchKernelGGL(k_adam, dim3(grid1(MLP_NPARAM)), dim3(256), 0, st, (int64_t)MLP_NPARAM, m.master,
                     m.grad, m.adam_m, m.adam_v, lr, b1, b2, eps, c1, c2);
  mlp_refresh_bf16(m, st);
}

void mlp_loss(int64_t n, const float* Y, const float* T, const double* Ahat, const int32_t* ahat_idx,
              int64_t nvalid, float* dY, float* row_loss, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_aloss, dim3(grid1(n, 128)), dim3(128), 0, st, n, Y, T, Ahat, ahat_idx, nvalid,
                       1.f / (float)std::max<int64_t>(nvalid, 1), dY, row_loss);
}

void mlp_gather(int64_t n, int64_t npad, const int32_t* idx, const uint16_t* X, const float* T,
                uint16_t* Xb, float* Tb, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_rows, dim3(grid1(npad * 64)), dim3(256), 0, st, n, npad, idx, X, T, Xb, Tb);
}

void block_features(int64_t nb, const int64_t* bptr, const int32_t* bdofs, const int64_t* Aptr,
                    const int32_t* Acol, const double* Aval, double eligible_max, uint16_t* X,
                    float* T, double* Ahat, double* dsq, int8_t* eligible, hipStream_t st) {
  if (nb > 0)
    hipLaunchKernelGGL(k_block_features, dim3(grid1(nb, 128)), dim3(128), 0, st, nb, bptr, bdofs, Aptr,
                       Acol, Aval, eligible_max, X, T, Ahat, dsq, eligible);
}

void refine_check(int64_t nb, const int64_t* bptr, const int8_t* eligible, const float* Y,
                  const double* Ahat, int steps, double tol, double* Wout, int8_t* accepted,
                  float* resid, hipStream_t st) {
  if (nb > 0)
    hipLaunchKernelGGL(k_refine_check, dim3(grid1(nb, 128)), dim3(128), 0, st, nb, bptr, eligible, Y,
                       Ahat, steps, tol, Wout, accepted, resid);
}

}  // namespace hamg
