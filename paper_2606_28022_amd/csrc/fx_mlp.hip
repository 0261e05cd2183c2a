// Learned initial monomer charges: features, bfloat16-weight perceptron
// (forward, gradient, Adam) and the fragment-wise projection of the guess.
// Layout of the weight vector: W1[64][20], b1[64], W2[64][64], b2[64],
// W3[2][64], b3[2].  All reductions run in a fixed order (no atomics).
#include <hip/hip_runtime.h>

#include "fx_device.hpp"
#include "fx_kernels.hpp"

namespace fx {

namespace mlp {
constexpr int NF = 20, H = 64, NO = 2;
constexpr int oW1 = 0, ob1 = oW1 + H * NF, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + NO * H;
constexpr int NW = ob3 + NO;
static_assert(NW == 5634, "weight vector size");
constexpr double RC = 6.0;                              // Angstrom
constexpr double ETA = 1.0 / (2.0 * 0.35 * 0.35);       // Angstrom^-2
constexpr double BOHR_A = 0.529177210903;
}  // namespace mlp

// round to the nearest bfloat16 (ties to even), kept as a float
__device__ inline float bf16r(float x) {
  unsigned u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// one-hot element (H, C, N, O) and 16 radial functions, one thread per real
// atom; source atoms staged in LDS 256 at a time; sums in FP64
__global__ void __launch_bounds__(256) k_mlp_features(DevSystem sys, float* out) {
  using namespace mlp;
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = sys.nreal;
  __shared__ double sx[256], sy[256], sz[256];
  double xa = 0, ya = 0, za = 0;
  if (A < N) {
    xa = sys.xyz[3 * A] * BOHR_A;
    ya = sys.xyz[3 * A + 1] * BOHR_A;
    za = sys.xyz[3 * A + 2] * BOHR_A;
  }
  double g[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) g[k] = 0.0;
  for (int b0 = 0; b0 < N; b0 += 256) {
    const int b = b0 + threadIdx.x;
    __syncthreads();
    if (b < N) {
      sx[threadIdx.x] = sys.xyz[3 * b] * BOHR_A;
      sy[threadIdx.x] = sys.xyz[3 * b + 1] * BOHR_A;
      sz[threadIdx.x] = sys.xyz[3 * b + 2] * BOHR_A;
    }
    __syncthreads();
    const int nb = min(256, N - b0);
    if (A < N)
      for (int k = 0; k < nb; ++k) {
        if (b0 + k == A) continue;
        const double dx = xa - sx[k], dy = ya - sy[k], dz = za - sz[k];
        const double R2 = dx * dx + dy * dy + dz * dz;
        if (R2 >= RC * RC) continue;
        const double R = sqrt(R2);
        const double fc = 0.5 * (cos(M_PI * R / RC) + 1.0);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const double rs = 0.5 + s * (5.5 / 15.0);
          g[s] += exp(-ETA * (R - rs) * (R - rs)) * fc;
        }
      }
  }
  if (A < N) {
    const int Z = sys.elems[sys.elem[A]].Z;
    float* o = out + (long long)A * NF;
    o[0] = Z == 1 ? 1.0f : 0.0f;
    o[1] = Z == 6 ? 1.0f : 0.0f;
    o[2] = Z == 7 ? 1.0f : 0.0f;
    o[3] = Z == 8 ? 1.0f : 0.0f;
#pragma unroll
    for (int s = 0; s < 16; ++s) o[4 + s] = (float)g[s];
  }
}

// forward pass, one thread per row; wr = bfloat16-rounded weights
__global__ void __launch_bounds__(256) k_mlp_forward(const float* wr, const float* X, float* Y, long long n) {
  using namespace mlp;
  __shared__ float w[NW];
  for (int i = threadIdx.x; i < NW; i += blockDim.x) w[i] = wr[i];
  __syncthreads();
  const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  float x[NF], h1[H];
#pragma unroll
  for (int f = 0; f < NF; ++f) x[f] = bf16r(X[a * NF + f]);
  for (int i = 0; i < H; ++i) {
    float v = w[ob1 + i];
#pragma unroll
    for (int f = 0; f < NF; ++f) v += w[oW1 + i * NF + f] * x[f];
    h1[i] = tanhf(v);
  }
  float y0 = w[ob3], y1 = w[ob3 + 1];
  for (int j = 0; j < H; ++j) {
    float v = w[ob2 + j];
#pragma unroll 16
    for (int i = 0; i < H; ++i) v += w[oW2 + j * H + i] * h1[i];
    const float h2 = tanhf(v);
    y0 += w[oW3 + j] * h2;
    y1 += w[oW3 + H + j] * h2;
  }
  Y[a * NO] = y0;
  Y[a * NO + 1] = y1;
}

// Loss and gradient of a tile of TA rows per work-group (written as one
// partial per work-group, reduced later in work-group order).
constexpr int TA = 32;
__global__ void __launch_bounds__(256)
    k_mlp_grad_partial(const float* wr, const float* X, const float* Yl, long long n, float* part,
                       double* loss_part) {
  using namespace mlp;
  __shared__ float w[NW];
  __shared__ float xs[TA][NF];
  __shared__ float h1[TA][H], h2[TA][H], dd[TA][H];
  __shared__ float dy[TA][NO];
  __shared__ double red[256];
  for (int i = threadIdx.x; i < NW; i += blockDim.x) w[i] = wr[i];
  const long long a0 = (long long)blockIdx.x * TA;
  for (int e = threadIdx.x; e < TA * NF; e += blockDim.x) {
    const int a = e / NF, f = e - a * NF;
    xs[a][f] = (a0 + a < n) ? bf16r(X[(a0 + a) * NF + f]) : 0.0f;
  }
  __syncthreads();
  // forward: hidden layers (row a, unit i)
  for (int e = threadIdx.x; e < TA * H; e += blockDim.x) {
    const int a = e / H, i = e - a * H;
    float v = w[ob1 + i];
    for (int f = 0; f < NF; ++f) v += w[oW1 + i * NF + f] * xs[a][f];
    h1[a][i] = tanhf(v);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TA * H; e += blockDim.x) {
    const int a = e / H, j = e - a * H;
    float v = w[ob2 + j];
    for (int i = 0; i < H; ++i) v += w[oW2 + j * H + i] * h1[a][i];
    h2[a][j] = tanhf(v);
  }
  __syncthreads();
  double lsum = 0.0;
  for (int e = threadIdx.x; e < TA * NO; e += blockDim.x) {
    const int a = e / NO, k = e - a * NO;
    float y = w[ob3 + k];
    for (int j = 0; j < H; ++j) y += w[oW3 + k * H + j] * h2[a][j];
    float g = 0.0f;
    if (a0 + a < n) {
      const float r = y - Yl[(a0 + a) * NO + k];
      lsum += (double)r * (double)r;
      g = 2.0f * r / (float)(n * NO);
    }
    dy[a][k] = g;
  }
  red[threadIdx.x] = lsum;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
  float* pg = part + (long long)blockIdx.x * NW;
  // output layer
  for (int e = threadIdx.x; e < NO * H + NO; e += blockDim.x) {
    if (e < NO * H) {
      const int k = e / H, j = e - k * H;
      float v = 0.0f;
      for (int a = 0; a < TA; ++a) v += dy[a][k] * h2[a][j];
      pg[oW3 + e] = v;
    } else {
      const int k = e - NO * H;
      float v = 0.0f;
      for (int a = 0; a < TA; ++a) v += dy[a][k];
      pg[ob3 + k] = v;
    }
  }
  // second hidden layer
  for (int e = threadIdx.x; e < TA * H; e += blockDim.x) {
    const int a = e / H, j = e - a * H;
    const float t = w[oW3 + j] * dy[a][0] + w[oW3 + H + j] * dy[a][1];
    dd[a][j] = t * (1.0f - h2[a][j] * h2[a][j]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < H * H + H; e += blockDim.x) {
    if (e < H * H) {
      const int j = e / H, i = e - j * H;
      float v = 0.0f;
      for (int a = 0; a < TA; ++a) v += dd[a][j] * h1[a][i];
      pg[oW2 + e] = v;
    } else {
      const int j = e - H * H;
      float v = 0.0f;
      for (int a = 0; a < TA; ++a) v += dd[a][j];
      pg[ob2 + j] = v;
    }
  }
  // first hidden layer (deltas into h2's storage)
  for (int e = threadIdx.x; e < TA * H; e += blockDim.x) {
    const int a = e / H, i = e - a * H;
    float t = 0.0f;
    for (int j = 0; j < H; ++j) t += dd[a][j] * w[oW2 + j * H + i];
    h2[a][i] = t * (1.0f - h1[a][i] * h1[a][i]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < H * NF + H; e += blockDim.x) {
    if (e < H * NF) {
      const int i = e / NF, f = e - i * NF;
      float v = 0.0f;
      for (int a = 0; a < TA; ++a) v += h2[a][i] * xs[a][f];
      pg[oW1 + e] = v;
    } else {
      const int i = e - H * NF;
      float v = 0.0f;
      for (int a = 0; a < TA; ++a) v += h2[a][i];
      pg[ob1 + i] = v;
    }
  }
}

// gradient = sum of the work-group partials in work-group order
__global__ void k_mlp_grad_reduce(const float* part, int nparts, float* grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mlp::NW) return;
  float v = 0.0f;
  for (int p = 0; p < nparts; ++p) v += part[(long long)p * mlp::NW + i];
  grad[i] = v;
}

__global__ void k_mlp_loss_reduce(const double* loss_part, int nparts, double inv_count, double* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double v = 0.0;
    for (int p = 0; p < nparts; ++p) v += loss_part[p];
    out[0] = v * inv_count;
  }
}

// Adam update of the FP32 master weights (step t >= 1) and their bfloat16
// rounding for the next forward pass
__global__ void k_mlp_adam(float* master, float* m, float* v, const float* g, int t, float lr, float* wr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mlp::NW) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[i] + (1.0f - b1) * g[i];
  const float vi = b2 * v[i] + (1.0f - b2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)t));
  const float vh = vi / (1.0f - powf(b2, (float)t));
  const float w = master[i] - lr * mh / (sqrtf(vh) + eps);
  master[i] = w;
  wr[i] = bf16r(w);
}

__global__ void k_mlp_round(const float* master, float* wr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < mlp::NW) wr[i] = bf16r(master[i]);
}

// guess of the global shell vector: the two predicted shell charges of each
// real atom, zero on ghost shells
__global__ void k_guess_assemble(DevSystem sys, const float* Y, double* q) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= sys.natoms) return;
  const int s0 = sys.atom_sh0[A], s1 = sys.atom_sh0[A + 1];
  for (int s = s0; s < s1; ++s) q[s] = (A < sys.nreal && s - s0 < 2) ? (double)Y[2 * A + (s - s0)] : 0.0;
}

// shift each fragment's real shells uniformly so that the fragment's shell
// charges (ghosts included) sum to minus its net charge; one work-group per
// fragment, fixed-order reduction
__global__ void k_guess_project(DevSystem sys, const int* frag_atoms, const int* frag_off, const int* frag_charge,
                                double* q) {
  const int I = blockIdx.x;
  __shared__ double red[256];
  __shared__ double cnt[256];
  double s = 0.0, c = 0.0;
  for (int ia = frag_off[I] + threadIdx.x; ia < frag_off[I + 1]; ia += blockDim.x) {
    const int A = frag_atoms[ia];
    for (int t = sys.atom_sh0[A]; t < sys.atom_sh0[A + 1]; ++t) {
      s += q[t];
      if (A < sys.nreal) c += 1.0;
    }
  }
  red[threadIdx.x] = s;
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      cnt[threadIdx.x] += cnt[threadIdx.x + w];
    }
    __syncthreads();
  }
  const double shift = (red[0] + (double)frag_charge[I]) / (cnt[0] > 0.0 ? cnt[0] : 1.0);
  for (int ia = frag_off[I] + threadIdx.x; ia < frag_off[I + 1]; ia += blockDim.x) {
    const int A = frag_atoms[ia];
    if (A >= sys.nreal) continue;
    for (int t = sys.atom_sh0[A]; t < sys.atom_sh0[A + 1]; ++t) q[t] -= shift;
  }
}

// restart from superposition charges: phase 0 after the first iteration for
// systems whose residual exceeds tau, phase 1 for systems still unconverged
__global__ void k_guess_fallback(DevBatch bt, const int* list, int nl, int phase, double tau, int* flag) {
  const int k = blockIdx.x;
  if (k >= nl) return;
  const int si = list[k];
  const SysDesc d = bt.desc[si];
  const bool reset = phase == 0 ? (tau > 0.0 && bt.err[si] > tau) : (bt.status[si] == 0);
  if (!reset) return;
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x) bt.q_in[d.sh_off + s] = 0.0;
  if (threadIdx.x == 0) {
    bt.nhist[si] = 0;
    bt.e_prev[si] = 0.0;
    flag[si] = 1;
  }
}

}  // namespace fx
