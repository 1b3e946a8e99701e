// icr_nn.hip -- warm-start network for the relaxation phase (not in the
// paper; it shortens the relaxation that the paper runs for 8 days before
// the period of interest, Sect. 3).
//
// Network (per sample): boundary map features X [n_theta][n_phi][8]
//   conv 3 x (phi_hi - phi_lo + 1) (periodic in phi, edge-clamped in theta) 8 -> C1, SiLU
//   conv 3x3 C1 -> C2, SiLU                              = latent z per column
//   per-column decoder: Linear C2 -> H, SiLU; Linear H -> n_r * 8
// output: normalised residual of the state over the radial expansion of the
// map.  All products run on BF16 MFMA (v_mfma_f32_32x32x16_bf16) with FP32
// accumulation; weights have FP32 masters updated by Adam and BF16 copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "icarus_nn.h"

namespace icrnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// float -> bf16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------------ GEMM --
// C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]), FP32 out, BF16 in.
// A(m,k) = TA ? a[k*lda + m] : a[m*lda + k];  B(k,n) = TB ? b[n*ldb + k] : b[k*ldb + n].
// Block tile 128 x 128 x 32, 4 waves of 64 x 64 (2 x 2 MFMA 32x32x16).
constexpr int BM = 128, BN = 128, BK = 32, KP = BK + 8;

template <int T>
__device__ __forceinline__ void load_tile(const uint16_t* __restrict__ g, int ld, int r0, int k0,
                                          int R, int K, uint16_t (*s)[KP]) {
  // s[r][k] for r in [0,128), k in [0,32): element (r0+r, k0+k) of a matrix
  // stored K-contiguous (T = 0: g[r*ld + k]) or R-contiguous (T = 1: g[k*ld + r]).
  const int tid = threadIdx.x;
  for (int c = tid; c < 512; c += 256) {
    if (T == 0) {
      const int r = c >> 2, kc = (c & 3) * 8;
      const int gr = r0 + r, gk = k0 + kc;
      uint16_t v[8];
      if (gr < R && gk + 8 <= K && (ld & 7) == 0) {
        const uint4 q = *reinterpret_cast<const uint4*>(g + (long long)gr * ld + gk);
        memcpy(v, &q, 16);
      } else {
        for (int i = 0; i < 8; ++i)
          v[i] = (gr < R && gk + i < K) ? g[(long long)gr * ld + gk + i] : (uint16_t)0;
      }
      memcpy(&s[r][kc], v, 16);
    } else {
      const int k = c >> 4, rc = (c & 15) * 8;
      const int gk = k0 + k, gr = r0 + rc;
      uint16_t v[8];
      if (gk < K && gr + 8 <= R && (ld & 7) == 0) {
        const uint4 q = *reinterpret_cast<const uint4*>(g + (long long)gk * ld + gr);
        memcpy(v, &q, 16);
      } else {
        for (int i = 0; i < 8; ++i)
          v[i] = (gk < K && gr + i < R) ? g[(long long)gk * ld + gr + i] : (uint16_t)0;
      }
      for (int i = 0; i < 8; ++i) s[rc + i][k] = v[i];
    }
  }
}

template <int TA, int TB>
__global__ void __launch_bounds__(256) k_gemm(const uint16_t* __restrict__ A,
                                              const uint16_t* __restrict__ B,
                                              float* __restrict__ C,
                                              const float* __restrict__ bias, int M, int N,
                                              int Kfull, int lda, int ldb, int ldc, int kchunk) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[BM][KP];
  __shared__ __attribute__((aligned(16))) uint16_t sB[BN][KP];
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  // split K: block z covers k in [z kchunk, min(K, (z + 1) kchunk)) and writes
  // its partial product to slab z of C (slabs M x ldc apart)
  const int kbeg = blockIdx.z * kchunk;
  const int K = Kfull < kbeg + kchunk ? Kfull : kbeg + kchunk;
  C += (long long)blockIdx.z * M * ldc;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  f32x16 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int q = 0; q < 16; ++q) acc[a][b][q] = 0.f;
  for (int k0 = kbeg; k0 < K; k0 += BK) {
    __syncthreads();
    load_tile<TA>(A, lda, m0, k0, M, K, sA);
    load_tile<TB ? 0 : 1>(B, ldb, n0, k0, N, K, sB);
    __syncthreads();
    for (int ks = 0; ks < BK; ks += 16) {
      const int kk = ks + (lane >> 5) * 8;
      bf16x8 fa[2], fb[2];
      for (int t = 0; t < 2; ++t) {
        memcpy(&fa[t], &sA[wm + t * 32 + (lane & 31)][kk], 16);
        memcpy(&fb[t], &sB[wn + t * 32 + (lane & 31)][kk], 16);
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
  }
  // accumulator element q = 4 i + j of a 32x32 tile holds row 8 i + 4 (lane / 32) + j,
  // column lane % 32
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int n = n0 + wn + b * 32 + (lane & 31);
      if (n >= N) continue;
      const float bn = bias ? bias[n] : 0.f;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          const int m = m0 + wm + a * 32 + 8 * i + 4 * (lane >> 5) + j;
          if (m < M) C[(long long)m * ldc + n] = acc[a][b][4 * i + j] + bn;
        }
    }
}

void gemm_launch(int ta, int tb, const uint16_t* A, const uint16_t* B, float* C,
                 const float* bias, int M, int N, int K, int lda, int ldb, int ldc, int splits,
                 int kchunk, hipStream_t s) {
  const dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, splits), blk(256);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<0, 0>), grid, blk, 0, s, A, B, C, bias, M, N, K, lda, ldb, ldc,
                       kchunk);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<0, 1>), grid, blk, 0, s, A, B, C, bias, M, N, K, lda, ldb, ldc,
                       kchunk);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<1, 0>), grid, blk, 0, s, A, B, C, bias, M, N, K, lda, ldb, ldc,
                       kchunk);
  else
    hipLaunchKernelGGL((k_gemm<1, 1>), grid, blk, 0, s, A, B, C, bias, M, N, K, lda, ldb, ldc,
                       kchunk);
}

void gemm(int ta, int tb, const uint16_t* A, const uint16_t* B, float* C, const float* bias, int M,
          int N, int K, int lda, int ldb, int ldc, hipStream_t s) {
  gemm_launch(ta, tb, A, B, C, bias, M, N, K, lda, ldb, ldc, 1, (K + BK - 1) / BK * BK, s);
}

// Split of the reduction dimension for products whose output has few tiles
// and whose K is long (the weight gradients, K = rows of the batch): enough
// (tile, slab) blocks to fill the chip, each slab a multiple of BK.
struct Split {
  int slabs, kchunk;
};
Split ksplit(int M, int N, int K) {
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int want = (1024 + tiles - 1) / tiles;
  const int most = (K + 8 * BK - 1) / (8 * BK);  // at least 8 k-steps per slab
  want = want < 1 ? 1 : (want > most ? most : want);
  const int kchunk = ((K + want - 1) / want + BK - 1) / BK * BK;
  return Split{(K + kchunk - 1) / kchunk, kchunk};
}

// C[i] = sum over slabs z (in order) of P[z][i]
__global__ void k_sum_slabs(const float* __restrict__ part, int slabs, long long n,
                            float* __restrict__ C) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int z = 0; z < slabs; ++z) acc += part[(long long)z * n + i];
  C[i] = acc;
}

// weight gradient C [M][N] (contiguous) from a product over a long K
void gemm_wgrad(int ta, int tb, const uint16_t* A, const uint16_t* B, float* C, int M, int N,
                int K, int lda, int ldb, float* scratch, hipStream_t s) {
  const Split sp = ksplit(M, N, K);
  if (sp.slabs == 1) {
    gemm(ta, tb, A, B, C, nullptr, M, N, K, lda, ldb, N, s);
    return;
  }
  gemm_launch(ta, tb, A, B, scratch, nullptr, M, N, K, lda, ldb, N, sp.slabs, sp.kchunk, s);
  const long long n = (long long)M * N;
  hipLaunchKernelGGL(k_sum_slabs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, scratch,
                     sp.slabs, n, C);
}

// ------------------------------------------------------------ elementwise --
__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// H = SiLU(Z) = Z / (1 + exp(-Z)) as BF16
__global__ void k_silu(const float* __restrict__ z, uint16_t* __restrict__ h, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const float v = z[i];
    h[i] = f2bf(v / (1.f + expf(-v)));
  }
}

// dZ = dH * SiLU'(Z), SiLU'(z) = s (1 + z (1 - s)), s = 1/(1+exp(-z)); FP32 and BF16 copies
__global__ void k_silu_back(const float* __restrict__ dh, const float* __restrict__ z,
                            float* __restrict__ dz, uint16_t* __restrict__ dzb, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const float v = z[i], s = 1.f / (1.f + expf(-v));
    const float d = dh[i] * s * (1.f + v * (1.f - s));
    dz[i] = d;
    dzb[i] = f2bf(d);
  }
}

// neighbourhood gather over 3 colatitude rows and nk longitudes starting at offset dk0:
// A[b, j, k][tap * C + c] = H[b, clamp(j + dj), (k + dk) mod np][c],
// tap = (dj + 1) * nk + (dk - dk0), dj in {-1, 0, 1}, dk in [dk0, dk0 + nk)
__global__ void k_im2col(const uint16_t* __restrict__ h, uint16_t* __restrict__ a, int B, int nt,
                         int np, int C, int dk0, int nk) {
  const int taps = 3 * nk;
  const long long n = (long long)B * nt * np * taps * C;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % C);
  long long r = i / C;
  const int tap = (int)(r % taps);
  r /= taps;
  const int k = (int)(r % np);
  r /= np;
  const int j = (int)(r % nt);
  const int b = (int)(r / nt);
  const int dj = tap / nk - 1, dk = tap % nk + dk0;
  int jj = j + dj;
  jj = jj < 0 ? 0 : (jj >= nt ? nt - 1 : jj);
  int kk = (k + dk) % np;
  if (kk < 0) kk += np;
  a[i] = h[(((long long)b * nt + jj) * np + kk) * C + c];
}

// adjoint of k_im2col: dH[b, j', k'][c] = sum of dA over every (j, k, tap) that gathered (j', k')
__global__ void k_col2im(const float* __restrict__ da, float* __restrict__ dh, int B, int nt,
                         int np, int C, int dk0, int nk) {
  const int taps = 3 * nk;
  const long long n = (long long)B * nt * np * C;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % C);
  long long r = i / C;
  const int k = (int)(r % np);
  r /= np;
  const int j = (int)(r % nt);
  const int b = (int)(r / nt);
  float s = 0.f;
  for (int dj = -1; dj <= 1; ++dj) {
    // source rows jsrc whose clamp(jsrc + dj) == j
    int js[2], ns = 0;
    const int j0 = j - dj;
    if (j0 >= 0 && j0 < nt) js[ns++] = j0;
    if (dj == -1 && j == 0) js[ns++] = 0;       // clamp(0 - 1) = 0
    if (dj == 1 && j == nt - 1) js[ns++] = nt - 1;  // clamp(nt - 1 + 1) = nt - 1
    for (int q = 0; q < ns; ++q)
      for (int t = 0; t < nk; ++t) {
        int ks = (k - (t + dk0)) % np;
        if (ks < 0) ks += np;
        const int tap = (dj + 1) * nk + t;
        s += da[((((long long)b * nt + js[q]) * np + ks) * taps + tap) * C + c];
      }
  }
  dh[i] = s;
}

// Column sums db[n] = sum_m dZ[m][n] in two passes with a fixed order:
// block (x, slab) sums rows of its slab for 64 columns (4 row phases per
// column, combined in order), then one thread per column adds the slabs.
constexpr int CS_SLABS = 64;
template <bool DIFF>
__global__ void __launch_bounds__(256) k_colsum_part(const float* __restrict__ a,
                                                     const float* __restrict__ b, int M, int N,
                                                     double* __restrict__ part) {
  __shared__ double sh[4][64];
  const int n = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
  const int rows = (M + CS_SLABS - 1) / CS_SLABS;
  const int m0 = blockIdx.y * rows, m1 = m0 + rows < M ? m0 + rows : M;
  double acc = 0.0;
  if (n < N)
    for (int m = m0 + ph; m < m1; m += 4) {
      const long long i = (long long)m * N + n;
      acc += DIFF ? (double)(a[i] - b[i]) : (double)a[i];
    }
  sh[ph][threadIdx.x & 63] = acc;
  __syncthreads();
  if (ph == 0 && n < N)
    part[(long long)blockIdx.y * N + n] = ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) +
                                           sh[2][threadIdx.x]) + sh[3][threadIdx.x];
}

__global__ void k_colsum_fin(const double* __restrict__ part, int N, double scale,
                             float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double acc = 0.0;
  for (int z = 0; z < CS_SLABS; ++z) acc += part[(long long)z * N + n];
  db[n] = (float)(acc * scale);
}

// db = scale * column sums of A (or of A - B when b != nullptr)
void colsum(const float* a, const float* b, int M, int N, double scale, float* db,
            double* scratch, hipStream_t s) {
  const dim3 grid((N + 63) / 64, CS_SLABS);
  if (b)
    hipLaunchKernelGGL(k_colsum_part<true>, grid, dim3(256), 0, s, a, b, M, N, scratch);
  else
    hipLaunchKernelGGL(k_colsum_part<false>, grid, dim3(256), 0, s, a, b, M, N, scratch);
  hipLaunchKernelGGL(k_colsum_fin, dim3((N + 255) / 256), dim3(256), 0, s, scratch, N, scale, db);
}

// dY = 2 (Y - T) / count (BF16 for the products), loss partial sums per block
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                      uint16_t* __restrict__ dy, double* __restrict__ part, long long n,
                      float scale) {
  __shared__ double sh[256];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    const float d = y[i] - t[i];
    dy[i] = f2bf(2.f * d * scale);
    e = (double)d * d;
  }
  sh[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out = sum of part[0..n): one block of 256, strided partial sums, then a
// fixed tree
__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ part, int n,
                                             double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Adam on FP32 masters, BF16 copies refreshed
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ pb, long long n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}

// ------------------------------------------------------ feature transforms --
struct Norm {
  double rho_ref, v_ref, p_ref, b_ref;
};

// X[b][j][k][f] from SI maps [b][8][nt][np] (cin = 8, or 10 with the two
// colatitude channels)
__global__ void k_encode_map(const double* __restrict__ maps, float* __restrict__ x, int B, int nt,
                             int np, double omega, double r_in, const double* __restrict__ thc,
                             Norm nz, int cin) {
  const long long n = (long long)B * nt * np;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int k = (int)(q % np);
  const int j = (int)((q / np) % nt);
  const int b = (int)(q / ((long long)nt * np));
  const long long plane = (long long)nt * np;
  const double* m = maps + (long long)b * 8 * plane + (long long)j * np + k;
  float* o = x + q * cin;
  if (cin > 8) {
    const double t = nt > 1 ? (2.0 * thc[j] - thc[0] - thc[nt - 1]) / (thc[nt - 1] - thc[0]) : 0.0;
    o[8] = (float)t;
    o[9] = (float)(2.0 * t * t - 1.0);
  }
  o[0] = (float)log(m[0] / nz.rho_ref);
  o[1] = (float)(m[1 * plane] / nz.v_ref - 5.0);
  o[2] = (float)(m[2 * plane] / nz.v_ref);
  o[3] = (float)((m[3 * plane] + omega * r_in * sin(thc[j])) / nz.v_ref);
  o[4] = (float)log(m[4 * plane] / nz.p_ref);
  o[5] = (float)(m[5 * plane] / nz.b_ref);
  o[6] = (float)(m[6 * plane] / nz.b_ref);
  o[7] = (float)(m[7 * plane] / nz.b_ref);
}

// radial expansion of the map column at r (same laws as the initial state)
__device__ __forceinline__ void radial_base(const double* m, long long plane, double r, double r_in,
                                            double omega, double sth, double gam, double (&w)[8]) {
  const double x = r_in / r;
  w[0] = m[0] * x * x;
  w[1] = m[plane];
  w[2] = 0.0;
  w[3] = -omega * r * sth;
  w[4] = m[4 * plane] * pow(x, 2.0 * gam);
  w[5] = m[5 * plane] * x * x;
  w[6] = 0.0;
  w[7] = m[7 * plane] * x;
}

// T[col][i*8 + v] (col = j*np + k) from a primitive SI state [8][np][nt][nr] and its map
__global__ void k_encode_target(const double* __restrict__ map, const double* __restrict__ st,
                                const double* __restrict__ rc, const double* __restrict__ thc,
                                float* __restrict__ t, int nr, int nt, int np, double omega,
                                double r_in, double gam, double v_ref) {
  const long long n = (long long)nr * nt * np;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int i = (int)(q % nr);
  const int j = (int)((q / nr) % nt);
  const int k = (int)(q / ((long long)nr * nt));
  const long long plane = (long long)nt * np;
  double w[8];
  radial_base(map + (long long)j * np + k, plane, rc[i], r_in, omega, sin(thc[j]), gam, w);
  const long long cell = ((long long)k * nt + j) * nr + i;
  double s[8];
  for (int v = 0; v < 8; ++v) s[v] = st[v * n + cell];
  const double bs = fabs(w[5]) + fabs(w[7]) + 1e-30;
  float* o = t + (((long long)j * np + k) * nr + i) * 8;
  o[0] = (float)log(s[0] / w[0]);
  o[1] = (float)((s[1] - w[1]) / v_ref);
  o[2] = (float)(s[2] / v_ref);
  o[3] = (float)((s[3] - w[3]) / v_ref);
  o[4] = (float)log(s[4] / w[4]);
  o[5] = (float)((s[5] - w[5]) / bs);
  o[6] = (float)(s[6] / bs);
  o[7] = (float)((s[7] - w[7]) / bs);
}

// inverse of k_encode_target: primitive SI state from the network output
__global__ void k_decode_state(const double* __restrict__ map, const float* __restrict__ y,
                               const double* __restrict__ rc, const double* __restrict__ thc,
                               double* __restrict__ st, int nr, int nt, int np, double omega,
                               double r_in, double gam, double v_ref) {
  const long long n = (long long)nr * nt * np;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int i = (int)(q % nr);
  const int j = (int)((q / nr) % nt);
  const int k = (int)(q / ((long long)nr * nt));
  const long long plane = (long long)nt * np;
  double w[8];
  radial_base(map + (long long)j * np + k, plane, rc[i], r_in, omega, sin(thc[j]), gam, w);
  const double bs = fabs(w[5]) + fabs(w[7]) + 1e-30;
  const float* o = y + (((long long)j * np + k) * nr + i) * 8;
  double s[8];
  s[0] = w[0] * exp((double)o[0]);
  s[1] = w[1] + v_ref * o[1];
  s[2] = v_ref * o[2];
  s[3] = w[3] + v_ref * o[3];
  s[4] = w[4] * exp((double)o[4]);
  s[5] = w[5] + bs * o[5];
  s[6] = bs * o[6];
  s[7] = w[7] + bs * o[7];
  const long long cell = ((long long)k * nt + j) * nr + i;
  for (int v = 0; v < 8; ++v) st[v * n + cell] = s[v];
}

}  // namespace icrnn

using namespace icrnn;

namespace {
thread_local std::string g_nn_err;
int nfail(int code, const char* fmt, ...) {
  char buf[400];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_nn_err = buf;
  return code;
}
#define NN_TRY(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return nfail(ICR_NN_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct Sizes {
  long long ncol, M;           // columns per sample, rows of a batch
  long long w1, w2, w3, w4;    // weight counts
  long long nparam;
  int cin, c1, c2, h, no, k1, k2;  // input features, channels, hidden, outputs, conv K
};

Sizes sizes(const icr_nn_shape& s) {
  Sizes z;
  z.ncol = (long long)s.n_theta * s.n_phi;
  z.M = z.ncol * s.batch_max;
  z.c1 = s.c1;
  z.c2 = s.c2;
  z.h = s.hidden;
  z.no = s.n_r * 8;
  z.cin = s.coord ? 10 : 8;
  z.k1 = 3 * (s.phi_hi - s.phi_lo + 1) * z.cin;
  z.k2 = 9 * s.c1;
  z.w1 = (long long)z.k1 * z.c1;
  z.w2 = (long long)z.k2 * z.c2;
  z.w3 = (long long)z.c2 * z.h;
  z.w4 = (long long)z.h * z.no;
  z.nparam = z.w1 + z.c1 + z.w2 + z.c2 + z.w3 + z.h + z.w4 + z.no;
  return z;
}

int check_shape(const icr_nn_shape* s) {
  if (!s) return nfail(ICR_NN_ERR_ARG, "shape is NULL");
  if (s->n_theta < 1 || s->n_phi < 3 || s->n_r < 1 || s->c1 < 1 || s->c2 < 1 || s->hidden < 1 ||
      s->batch_max < 1 || (s->coord != 0 && s->coord != 1))
    return nfail(ICR_NN_ERR_ARG, "invalid network shape");
  if (s->phi_lo > 0 || s->phi_hi < 0 || s->phi_hi - s->phi_lo + 1 > s->n_phi)
    return nfail(ICR_NN_ERR_ARG, "first-layer longitude window must hold offset 0 and fit n_phi");
  return ICR_NN_OK;
}

}  // namespace

struct icr_nn {
  icr_nn_shape s;
  Sizes z;
  hipStream_t stream;
  char* ws;
  // parameters: fp32 master, bf16 copy, grads, Adam moments (same layout)
  float *p, *g, *m, *v;
  uint16_t* pb;
  long long step;
  // activations (batch_max rows)
  float *x;                                // [M][8] features
  uint16_t *xb, *a1, *h1, *a2, *h2, *h3;   // bf16 operands
  float *z1, *z2, *z3, *y;                 // pre-activations and output
  uint16_t *dyb, *dz3b, *dz2b, *dz1b;
  float *dh3, *dz3, *dh2, *dz2, *da2, *dh1, *dz1;
  double *part, *loss;
  float* split;    // split-K partial products of the weight gradients
  double* cpart;   // column-sum partials [CS_SLABS][widest layer]
  // parameter views
  float *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
  uint16_t *W1b, *W2b, *W3b, *W4b;
  float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3, *gW4, *gb4;
};

namespace {

size_t layout(const icr_nn_shape& s, icr_nn* n) {
  const Sizes z = sizes(s);
  size_t off = 0;
  char* base = n ? n->ws : nullptr;
  auto take = [&](size_t b) {
    char* p = base ? base + off : nullptr;
    off += al(b);
    return p;
  };
  const long long P = z.nparam, M = z.M;
  float* p = (float*)take(4 * P);
  float* g = (float*)take(4 * P);
  float* m = (float*)take(4 * P);
  float* v = (float*)take(4 * P);
  uint16_t* pb = (uint16_t*)take(2 * P);
  float* x = (float*)take(4 * M * z.cin);
  uint16_t* xb = (uint16_t*)take(2 * M * z.cin);
  uint16_t* a1 = (uint16_t*)take(2 * M * z.k1);
  float* z1 = (float*)take(4 * M * z.c1);
  uint16_t* h1 = (uint16_t*)take(2 * M * z.c1);
  uint16_t* a2 = (uint16_t*)take(2 * M * z.k2);
  float* z2 = (float*)take(4 * M * z.c2);
  uint16_t* h2 = (uint16_t*)take(2 * M * z.c2);
  float* z3 = (float*)take(4 * M * z.h);
  uint16_t* h3 = (uint16_t*)take(2 * M * z.h);
  float* y = (float*)take(4 * M * z.no);
  uint16_t* dyb = (uint16_t*)take(2 * M * z.no);
  float* dh3 = (float*)take(4 * M * z.h);
  float* dz3 = (float*)take(4 * M * z.h);
  uint16_t* dz3b = (uint16_t*)take(2 * M * z.h);
  float* dh2 = (float*)take(4 * M * z.c2);
  float* dz2 = (float*)take(4 * M * z.c2);
  uint16_t* dz2b = (uint16_t*)take(2 * M * z.c2);
  float* da2 = (float*)take(4 * M * z.k2);
  float* dh1 = (float*)take(4 * M * z.c1);
  float* dz1 = (float*)take(4 * M * z.c1);
  uint16_t* dz1b = (uint16_t*)take(2 * M * z.c1);
  const long long nblk = (M * z.no + 255) / 256;
  double* part = (double*)take(8 * nblk);
  double* loss = (double*)take(8);
  long long nsplit = 1;
  {
    const int dims[4][2] = {{z.h, z.no}, {z.c2, z.h}, {z.k2, z.c2}, {z.k1, z.c1}};
    for (const auto& d : dims) {
      const Split sp = ksplit(d[0], d[1], (int)M);
      if (sp.slabs > 1 && (long long)sp.slabs * d[0] * d[1] > nsplit)
        nsplit = (long long)sp.slabs * d[0] * d[1];
    }
  }
  float* split = (float*)take(4 * nsplit);
  int wmax = z.no > z.h ? z.no : z.h;
  wmax = wmax > z.c2 ? wmax : z.c2;
  wmax = wmax > z.c1 ? wmax : z.c1;
  double* cpart = (double*)take(8LL * CS_SLABS * wmax);
  if (n) {
    n->z = z;
    n->p = p; n->g = g; n->m = m; n->v = v; n->pb = pb;
    n->x = x; n->xb = xb; n->a1 = a1; n->z1 = z1; n->h1 = h1; n->a2 = a2; n->z2 = z2;
    n->h2 = h2; n->z3 = z3; n->h3 = h3; n->y = y; n->dyb = dyb; n->dh3 = dh3; n->dz3 = dz3;
    n->dz3b = dz3b; n->dh2 = dh2; n->dz2 = dz2; n->dz2b = dz2b; n->da2 = da2; n->dh1 = dh1;
    n->dz1 = dz1; n->dz1b = dz1b; n->part = part; n->loss = loss; n->split = split;
    n->cpart = cpart;
    long long o = 0;
    auto view = [&](long long cnt, float*& fp, float*& gp, uint16_t** bp) {
      fp = p + o;
      gp = g + o;
      if (bp) *bp = pb + o;
      o += cnt;
    };
    view(z.w1, n->W1, n->gW1, &n->W1b);
    view(z.c1, n->b1, n->gb1, nullptr);
    view(z.w2, n->W2, n->gW2, &n->W2b);
    view(z.c2, n->b2, n->gb2, nullptr);
    view(z.w3, n->W3, n->gW3, &n->W3b);
    view(z.h, n->b3, n->gb3, nullptr);
    view(z.w4, n->W4, n->gW4, &n->W4b);
    view(z.no, n->b4, n->gb4, nullptr);
  }
  return off;
}

inline dim3 g1(long long n) { return dim3((unsigned)((n + 255) / 256)); }

void forward(icr_nn* n, int B, const float* x_dev) {
  const Sizes& z = n->z;
  const int nt = n->s.n_theta, np = n->s.n_phi;
  const long long M = (long long)B * z.ncol;
  hipStream_t s = n->stream;
  hipLaunchKernelGGL(k_to_bf16, g1(M * z.cin), dim3(256), 0, s, x_dev, n->xb, M * z.cin);
  hipLaunchKernelGGL(k_im2col, g1(M * z.k1), dim3(256), 0, s, n->xb, n->a1, B, nt, np, z.cin,
                     n->s.phi_lo, n->s.phi_hi - n->s.phi_lo + 1);
  gemm(0, 0, n->a1, n->W1b, n->z1, n->b1, (int)M, z.c1, z.k1, z.k1, z.c1, z.c1, s);
  hipLaunchKernelGGL(k_silu, g1(M * z.c1), dim3(256), 0, s, n->z1, n->h1, M * z.c1);
  hipLaunchKernelGGL(k_im2col, g1(M * z.k2), dim3(256), 0, s, n->h1, n->a2, B, nt, np, z.c1,
                     -1, 3);
  gemm(0, 0, n->a2, n->W2b, n->z2, n->b2, (int)M, z.c2, z.k2, z.k2, z.c2, z.c2, s);
  hipLaunchKernelGGL(k_silu, g1(M * z.c2), dim3(256), 0, s, n->z2, n->h2, M * z.c2);
  gemm(0, 0, n->h2, n->W3b, n->z3, n->b3, (int)M, z.h, z.c2, z.c2, z.h, z.h, s);
  hipLaunchKernelGGL(k_silu, g1(M * z.h), dim3(256), 0, s, n->z3, n->h3, M * z.h);
  gemm(0, 0, n->h3, n->W4b, n->y, n->b4, (int)M, z.no, z.h, z.h, z.no, z.no, s);
}

void backward(icr_nn* n, int B, const float* t_dev) {
  const Sizes& z = n->z;
  const int nt = n->s.n_theta, np = n->s.n_phi;
  const long long M = (long long)B * z.ncol;
  hipStream_t s = n->stream;
  const long long ny = M * z.no;
  const int nblk = (int)((ny + 255) / 256);
  hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, n->y, t_dev, n->dyb, n->part, ny,
                     1.f / (float)ny);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, n->part, nblk, n->loss);
  // decoder layer 2: Y = H3 W4 + b4
  gemm_wgrad(1, 0, n->h3, n->dyb, n->gW4, z.h, z.no, (int)M, z.h, z.no, n->split, s);
  // db4 = colsum(dY) needs dY in FP32: recompute as 2(Y - T)/ny inside a colsum of Y - T
  gemm(0, 1, n->dyb, n->W4b, n->dh3, nullptr, (int)M, z.h, z.no, z.no, z.no, z.h, s);
  hipLaunchKernelGGL(k_silu_back, g1(M * z.h), dim3(256), 0, s, n->dh3, n->z3, n->dz3, n->dz3b,
                     M * z.h);
  gemm_wgrad(1, 0, n->h2, n->dz3b, n->gW3, z.c2, z.h, (int)M, z.c2, z.h, n->split, s);
  colsum(n->dz3, nullptr, (int)M, z.h, 1.0, n->gb3, n->cpart, s);
  gemm(0, 1, n->dz3b, n->W3b, n->dh2, nullptr, (int)M, z.c2, z.h, z.h, z.h, z.c2, s);
  hipLaunchKernelGGL(k_silu_back, g1(M * z.c2), dim3(256), 0, s, n->dh2, n->z2, n->dz2, n->dz2b,
                     M * z.c2);
  gemm_wgrad(1, 0, n->a2, n->dz2b, n->gW2, z.k2, z.c2, (int)M, z.k2, z.c2, n->split, s);
  colsum(n->dz2, nullptr, (int)M, z.c2, 1.0, n->gb2, n->cpart, s);
  gemm(0, 1, n->dz2b, n->W2b, n->da2, nullptr, (int)M, z.k2, z.c2, z.c2, z.c2, z.k2, s);
  hipLaunchKernelGGL(k_col2im, g1(M * z.c1), dim3(256), 0, s, n->da2, n->dh1, B, nt, np, z.c1,
                     -1, 3);
  hipLaunchKernelGGL(k_silu_back, g1(M * z.c1), dim3(256), 0, s, n->dh1, n->z1, n->dz1, n->dz1b,
                     M * z.c1);
  gemm_wgrad(1, 0, n->a1, n->dz1b, n->gW1, z.k1, z.c1, (int)M, z.k1, z.c1, n->split, s);
  colsum(n->dz1, nullptr, (int)M, z.c1, 1.0, n->gb1, n->cpart, s);
}

}  // namespace


extern "C" {

const char* icr_nn_last_error(void) { return g_nn_err.c_str(); }

int icr_nn_param_count(const icr_nn_shape* s, long long* n) {
  int rc = check_shape(s);
  if (rc) return rc;
  if (!n) return nfail(ICR_NN_ERR_ARG, "n is NULL");
  *n = sizes(*s).nparam;
  return ICR_NN_OK;
}

int icr_nn_workspace_bytes(const icr_nn_shape* s, size_t* bytes) {
  int rc = check_shape(s);
  if (rc) return rc;
  if (!bytes) return nfail(ICR_NN_ERR_ARG, "bytes is NULL");
  *bytes = layout(*s, nullptr);
  return ICR_NN_OK;
}

int icr_nn_create(const icr_nn_shape* s, void* ws, size_t bytes, void* stream, icr_nn** out) {
  int rc = check_shape(s);
  if (rc) return rc;
  if (!out) return nfail(ICR_NN_ERR_ARG, "out is NULL");
  const size_t need = layout(*s, nullptr);
  if (!ws || bytes < need) return nfail(ICR_NN_ERR_ARG, "workspace too small (%zu < %zu)", bytes, need);
  if (((uintptr_t)ws & 255) != 0) return nfail(ICR_NN_ERR_ARG, "workspace must be 256-byte aligned");
  icr_nn* n = new icr_nn();
  n->s = *s;
  n->stream = (hipStream_t)stream;
  n->ws = (char*)ws;
  n->step = 0;
  layout(*s, n);
  *out = n;
  return ICR_NN_OK;
}

void icr_nn_destroy(icr_nn* n) { delete n; }

int icr_nn_set_params(icr_nn* n, const float* host) {
  if (!n || !host) return nfail(ICR_NN_ERR_ARG, "NULL argument");
  const long long P = n->z.nparam;
  NN_TRY(hipMemcpyAsync(n->p, host, 4 * P, hipMemcpyHostToDevice, n->stream));
  NN_TRY(hipMemsetAsync(n->m, 0, 4 * P, n->stream));
  NN_TRY(hipMemsetAsync(n->v, 0, 4 * P, n->stream));
  hipLaunchKernelGGL(k_to_bf16, g1(P), dim3(256), 0, n->stream, n->p, n->pb, P);
  NN_TRY(hipStreamSynchronize(n->stream));
  n->step = 0;
  return ICR_NN_OK;
}

int icr_nn_get_params(icr_nn* n, float* host) {
  if (!n || !host) return nfail(ICR_NN_ERR_ARG, "NULL argument");
  NN_TRY(hipMemcpyAsync(host, n->p, 4 * n->z.nparam, hipMemcpyDeviceToHost, n->stream));
  NN_TRY(hipStreamSynchronize(n->stream));
  return ICR_NN_OK;
}

int icr_nn_forward(icr_nn* n, int batch, const float* x_dev, float* y_dev) {
  if (!n || !x_dev) return nfail(ICR_NN_ERR_ARG, "NULL argument");
  if (batch < 1 || batch > n->s.batch_max) return nfail(ICR_NN_ERR_ARG, "batch outside [1, %d]", n->s.batch_max);
  forward(n, batch, x_dev);
  if (y_dev) {
    const long long ny = (long long)batch * n->z.ncol * n->z.no;
    NN_TRY(hipMemcpyAsync(y_dev, n->y, 4 * ny, hipMemcpyDeviceToDevice, n->stream));
  }
  NN_TRY(hipGetLastError());
  return ICR_NN_OK;
}

int icr_nn_loss_grad(icr_nn* n, int batch, const float* x_dev, const float* t_dev, double* loss,
                     float* grad_host) {
  if (!n || !x_dev || !t_dev) return nfail(ICR_NN_ERR_ARG, "NULL argument");
  if (batch < 1 || batch > n->s.batch_max) return nfail(ICR_NN_ERR_ARG, "batch outside [1, %d]", n->s.batch_max);
  forward(n, batch, x_dev);
  backward(n, batch, t_dev);
  const long long M = (long long)batch * n->z.ncol;
  const long long ny = M * n->z.no;
  colsum(n->y, t_dev, (int)M, n->z.no, 2.0 / (double)ny, n->gb4, n->cpart, n->stream);
  NN_TRY(hipGetLastError());
  double l = 0.0;
  NN_TRY(hipMemcpyAsync(&l, n->loss, 8, hipMemcpyDeviceToHost, n->stream));
  if (grad_host)
    NN_TRY(hipMemcpyAsync(grad_host, n->g, 4 * n->z.nparam, hipMemcpyDeviceToHost, n->stream));
  NN_TRY(hipStreamSynchronize(n->stream));
  if (loss) *loss = l / (double)ny;
  return ICR_NN_OK;
}

int icr_nn_adam_step(icr_nn* n, float lr, float beta1, float beta2, float eps) {
  if (!n) return nfail(ICR_NN_ERR_ARG, "NULL argument");
  n->step += 1;
  const float c1 = 1.f - powf(beta1, (float)n->step), c2 = 1.f - powf(beta2, (float)n->step);
  hipLaunchKernelGGL(k_adam, g1(n->z.nparam), dim3(256), 0, n->stream, n->p, n->g, n->m, n->v,
                     n->pb, n->z.nparam, lr, beta1, beta2, eps, c1, c2);
  NN_TRY(hipGetLastError());
  return ICR_NN_OK;
}

int icr_nn_encode_map(icr_nn* n, int batch, const double* maps_dev, const double* thc_dev,
                      double omega, double r_in, float* x_dev) {
  if (!n || !maps_dev || !thc_dev || !x_dev) return nfail(ICR_NN_ERR_ARG, "NULL argument");
  const Norm nz{1.67262192369e-27 * 1e8, 1e5, 2.0 * 1e8 * 1.380649e-23 * 1e6, 250e-9};
  const long long q = (long long)batch * n->z.ncol;
  hipLaunchKernelGGL(k_encode_map, g1(q), dim3(256), 0, n->stream, maps_dev, x_dev, batch,
                     n->s.n_theta, n->s.n_phi, omega, r_in, thc_dev, nz, n->z.cin);
  NN_TRY(hipGetLastError());
  return ICR_NN_OK;
}

int icr_nn_encode_target(icr_nn* n, const double* map_dev, const double* state_dev,
                         const double* rc_dev, const double* thc_dev, double omega, double r_in,
                         double gamma, float* t_dev) {
  if (!n || !map_dev || !state_dev || !rc_dev || !thc_dev || !t_dev)
    return nfail(ICR_NN_ERR_ARG, "NULL argument");
  const long long c = (long long)n->s.n_r * n->z.ncol;
  hipLaunchKernelGGL(k_encode_target, g1(c), dim3(256), 0, n->stream, map_dev, state_dev, rc_dev,
                     thc_dev, t_dev, n->s.n_r, n->s.n_theta, n->s.n_phi, omega, r_in, gamma, 1e5);
  NN_TRY(hipGetLastError());
  return ICR_NN_OK;
}

int icr_nn_decode_state(icr_nn* n, const double* map_dev, const float* y_dev, const double* rc_dev,
                        const double* thc_dev, double omega, double r_in, double gamma,
                        double* state_dev) {
  if (!n || !map_dev || !y_dev || !rc_dev || !thc_dev || !state_dev)
    return nfail(ICR_NN_ERR_ARG, "NULL argument");
  const long long c = (long long)n->s.n_r * n->z.ncol;
  hipLaunchKernelGGL(k_decode_state, g1(c), dim3(256), 0, n->stream, map_dev, y_dev, rc_dev,
                     thc_dev, state_dev, n->s.n_r, n->s.n_theta, n->s.n_phi, omega, r_in, gamma,
                     1e5);
  NN_TRY(hipGetLastError());
  return ICR_NN_OK;
}

int icr_nn_gemm_bf16(int trans_a, int trans_b, int M, int N, int K, const void* A, int lda,
                     const void* B, int ldb, float* C, int ldc, const float* bias, void* stream) {
  if (M < 1 || N < 1 || K < 1 || !A || !B || !C) return nfail(ICR_NN_ERR_ARG, "invalid GEMM");
  gemm(trans_a, trans_b, (const uint16_t*)A, (const uint16_t*)B, C, bias, M, N, K, lda, ldb, ldc,
       (hipStream_t)stream);
  NN_TRY(hipGetLastError());
  return ICR_NN_OK;
}

}  // extern "C"
