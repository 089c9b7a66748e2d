// Learned d0 / rank predictor: a fully connected ReLU network in FP32.
//
// One workgroup (4 waves) owns a tile of 32 samples.  All activations of
// the tile stay in LDS, row-major with an odd leading dimension; every
// product (forward Z = H W^T, weight gradient G = Delta^T H, backward
// Delta W) runs on v_mfma_f32_16x16x4f32 with the waves taking 16x16
// output tiles round-robin.  Backward overwrites each hidden activation
// tile with its delta once the weight gradient that needs it is done, so
// the LDS footprint is one tile per layer boundary.
//
// Per-workgroup weight/bias gradients go to a partial buffer; a second
// kernel sums the partials in workgroup order (deterministic), scales by
// 2 / (number of unmasked targets) and optionally applies Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hss_internal.h"

namespace hss {

typedef float mflt4 __attribute__((ext_vector_type(4)));

constexpr int MLP_TILE = 32;
constexpr int MLP_THREADS = 256;

// C(M x N) = sum_k A(m, k) B(k, n).  Operand layouts of the FP32 16x16x4
// MFMA: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; the result
// element v of lane l is C[4 (l / 16) + v][l % 16].
template <class FA, class FB, class FS>
__device__ __forceinline__ void wave_mm(int M, int N, int K, FA A, FB B, FS store) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
  for (int t = wave; t < tm * tn; t += nw) {
    const int m0 = (t % tm) << 4, n0 = (t / tm) << 4;
    const int am = m0 + (lane & 15), bn = n0 + (lane & 15);
    mflt4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + (lane >> 4);
      const float a = (am < M && k < K) ? A(am, k) : 0.f;
      const float b = (bn < N && k < K) ? B(k, bn) : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = m0 + 4 * (lane >> 4) + v;
      if (r < M && bn < N) store(r, bn, acc[v]);
    }
  }
}

__device__ __forceinline__ int64_t mlp_row(int64_t pos, int64_t pa, int64_t pc, int64_t nd) {
  return (pa * pos + pc) % nd;
}

// mode 0: forward only, Y[row] = network(X[row]).
// mode 1: forward + backward; partial gradients to part[blockIdx.x][np],
//         (mask count, squared-error sum) to cl[2 blockIdx.x ..].
// Tile row s holds position p0 + s of the (affinely permuted) sample order;
// data row = (pa * position + pc) mod n_data.
__global__ __launch_bounds__(MLP_THREADS) void k_mlp_tile(MlpShape S, const float* __restrict__ P,
                                                          const float* __restrict__ X,
                                                          const float* __restrict__ T,
                                                          const float* __restrict__ Mk, int64_t pos0,
                                                          int64_t pos1, int64_t pa, int64_t pc, int64_t nd,
                                                          float* __restrict__ Y, float* __restrict__ part,
                                                          float* __restrict__ cl, int32_t mode) {
  extern __shared__ float lds[];
  const int tid = threadIdx.x;
  const int64_t p0 = pos0 + (int64_t)blockIdx.x * MLP_TILE;
  const int nrow = (int)min<int64_t>(MLP_TILE, pos1 - p0);
  const int nl = S.nl;

  {
    const int in = S.sz[0], ld = S.ald[0];
    float* A0 = lds + S.aoff[0];
    for (int idx = tid; idx < MLP_TILE * in; idx += blockDim.x) {
      const int s = idx / in, k = idx - s * in;
      A0[s * ld + k] = s < nrow ? X[mlp_row(p0 + s, pa, pc, nd) * in + k] : 0.f;
    }
  }
  __syncthreads();

  for (int l = 0; l < nl; ++l) {
    const int in = S.sz[l], out = S.sz[l + 1];
    const int ldi = S.ald[l], ldo = S.ald[l + 1];
    const float* W = P + S.woff[l];
    const float* bias = P + S.boff[l];
    const float* Ain = lds + S.aoff[l];
    float* Aout = lds + S.aoff[l + 1];
    const bool hidden = l < nl - 1;
    wave_mm(
        MLP_TILE, out, in, [&](int s, int k) { return Ain[s * ldi + k]; },
        [&](int k, int o) { return W[(int64_t)o * in + k]; },
        [&](int s, int o, float v) {
          v += bias[o];
          Aout[s * ldo + o] = hidden ? fmaxf(v, 0.f) : v;
        });
    __syncthreads();
  }

  const int out = S.sz[nl], ldy = S.ald[nl];
  float* Ay = lds + S.aoff[nl];
  if (mode == 0) {
    for (int idx = tid; idx < MLP_TILE * out; idx += blockDim.x) {
      const int s = idx / out, o = idx - s * out;
      if (s < nrow) Y[mlp_row(p0 + s, pa, pc, nd) * out + o] = Ay[s * ldy + o];
    }
    return;
  }

  // output delta (without the 2 / count factor, applied in the reduction)
  __shared__ float red[2][MLP_THREADS / 64];
  float lsum = 0.f, csum = 0.f;
  for (int idx = tid; idx < MLP_TILE * out; idx += blockDim.x) {
    const int s = idx / out, o = idx - s * out;
    float dlt = 0.f;
    if (s < nrow) {
      const int64_t r = mlp_row(p0 + s, pa, pc, nd);
      const float m = Mk[r * out + o];
      const float e = Ay[s * ldy + o] - T[r * out + o];
      dlt = m * e;
      lsum += m * e * e;
      csum += m;
    }
    Ay[s * ldy + o] = dlt;
  }
  for (int off = 32; off > 0; off >>= 1) {
    lsum += __shfl_down(lsum, off, 64);
    csum += __shfl_down(csum, off, 64);
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = csum;
    red[1][tid >> 6] = lsum;
  }
  __syncthreads();
  if (tid == 0) {
    float c = 0.f, q = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      c += red[0][w];
      q += red[1][w];
    }
    cl[2 * (int64_t)blockIdx.x] = c;
    cl[2 * (int64_t)blockIdx.x + 1] = q;
  }

  float* G = part + (int64_t)blockIdx.x * S.np;
  for (int l = nl - 1; l >= 0; --l) {
    const int in = S.sz[l], o_n = S.sz[l + 1];
    const int ldi = S.ald[l], ldo = S.ald[l + 1];
    const float* W = P + S.woff[l];
    float* H = lds + S.aoff[l];
    const float* Dl = lds + S.aoff[l + 1];
    float* GW = G + S.woff[l];
    wave_mm(
        o_n, in, MLP_TILE, [&](int o, int s) { return Dl[s * ldo + o]; },
        [&](int s, int i) { return H[s * ldi + i]; },
        [&](int o, int i, float v) { GW[(int64_t)o * in + i] = v; });
    for (int o = tid; o < o_n; o += blockDim.x) {
      float b = 0.f;
      for (int s = 0; s < MLP_TILE; ++s) b += Dl[s * ldo + o];
      G[S.boff[l] + o] = b;
    }
    __syncthreads();
    if (l > 0) {
      // delta_{l}[s][i] = (sum_o delta_{l+1}[s][o] W[o][i]) * [h_l[s][i] > 0], in place over h_l
      wave_mm(
          MLP_TILE, in, o_n, [&](int s, int o) { return Dl[s * ldo + o]; },
          [&](int o, int i) { return W[(int64_t)o * in + i]; },
          [&](int s, int i, float v) { H[s * ldi + i] = H[s * ldi + i] > 0.f ? v : 0.f; });
      __syncthreads();
    }
  }
}

__device__ __forceinline__ void adam_update(float& p, float g, float& m, float& v, const MlpAdam& a) {
  m = a.b1 * m + (1.f - a.b1) * g;
  v = a.b2 * v + (1.f - a.b2) * g * g;
  p -= a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
}

// Sum the per-workgroup partial gradients in workgroup order, scale by
// 2 / max(1, count); write the gradient and/or take one Adam step.
__global__ __launch_bounds__(256) void k_mlp_reduce(int64_t np, int32_t nblk, const float* __restrict__ part,
                                                    const float* __restrict__ cl, float* __restrict__ grad,
                                                    float* __restrict__ loss_out, float* __restrict__ params,
                                                    float* __restrict__ am, float* __restrict__ av, MlpAdam a,
                                                    int32_t adam) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float cnt = 0.f;
  for (int w = 0; w < nblk; ++w) cnt += cl[2 * w];
  const float scale = 2.f / fmaxf(1.f, cnt);
  if (p < np) {
    float g = 0.f;
    for (int w = 0; w < nblk; ++w) g += part[(int64_t)w * np + p];
    g *= scale;
    if (grad) grad[p] = g;
    if (adam) adam_update(params[p], g, am[p], av[p], a);
  }
  if (p == 0 && loss_out) {
    float q = 0.f;
    for (int w = 0; w < nblk; ++w) q += cl[2 * w + 1];
    *loss_out = q / fmaxf(1.f, cnt);
  }
}

__global__ __launch_bounds__(256) void k_mlp_adam(int64_t np, float* __restrict__ params,
                                                  const float* __restrict__ grad, float* __restrict__ am,
                                                  float* __restrict__ av, MlpAdam a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) adam_update(params[p], grad[p], am[p], av[p], a);
}

MlpShape mlp_shape(const hss_mlp& net) {
  if (net.n_layers < 1 || net.n_layers > HSS_MLP_MAX_LAYERS)
    throw Error(HSS_ERR_INVALID_ARG, "n_layers must be in [1, HSS_MLP_MAX_LAYERS]");
  MlpShape S{};
  S.nl = net.n_layers;
  int64_t off = 0;
  int32_t lo = 0;
  for (int l = 0; l <= S.nl; ++l) {
    const int w = net.sizes[l];
    if (w < 1 || w > HSS_MLP_MAX_WIDTH) throw Error(HSS_ERR_INVALID_ARG, "layer widths must be in [1, 128]");
    S.sz[l] = w;
    S.ald[l] = w | 1;  // odd leading dimension
    S.aoff[l] = lo;
    lo += MLP_TILE * S.ald[l];
  }
  for (int l = 0; l < S.nl; ++l) {
    S.woff[l] = off;
    off += (int64_t)S.sz[l + 1] * S.sz[l];
    S.boff[l] = off;
    off += S.sz[l + 1];
  }
  S.np = off;
  S.lds_floats = lo;
  if ((size_t)lo * sizeof(float) > 64 * 1024)
    throw Error(HSS_ERR_INVALID_ARG, "network activations of one tile exceed 64 KiB of LDS");
  return S;
}

int64_t mlp_tiles(int64_t rows) { return (rows + MLP_TILE - 1) / MLP_TILE; }

void launch_mlp_tile(const MlpShape& S, const float* P, const float* X, const float* T, const float* M,
                     int64_t pos0, int64_t pos1, int64_t pa, int64_t pc, int64_t nd, float* Y, float* part,
                     float* cl, int mode, hipStream_t s) {
  const int64_t nb = mlp_tiles(pos1 - pos0);
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_mlp_tile, dim3((unsigned)nb), dim3(MLP_THREADS), S.lds_floats * sizeof(float), s, S, P,
                     X, T, M, pos0, pos1, pa, pc, nd, Y, part, cl, mode);
}

void launch_mlp_reduce(int64_t np, int32_t nblk, const float* part, const float* cl, float* grad, float* loss,
                       float* params, float* am, float* av, const MlpAdam& a, int adam, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np, nblk, part, cl,
                     grad, loss, params, am, av, a, adam);
}

void launch_mlp_adam(int64_t np, float* params, const float* grad, float* am, float* av, const MlpAdam& a,
                     hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np, params, grad, am, av,
                     a);
}

}  // namespace hss
