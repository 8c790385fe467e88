// Learned warm start for the Newton iteration (gfx950).
//
// The Newton iteration of Supplement section 2.3 starts from lambda_0 = 0.
// Here a small network predicts lambda_0 from local constraint geometry:
// per constraint k a 16-feature vector (rotation, translation and
// mass-scale invariant: the decoupled diatomic solution t0_k, the initial
// violation, geometry of old vs unconstrained bond vector, valences, and
// sums over the constraints sharing an atom weighted by the normalised
// coupling rho_kj = A_kj(r, r) / A_kk(r, r) of Eq. defA) feeds an MLP
// [16 -> 64 -> 64 -> 1] with exact GELU whose output corrects t0:
//   lambda_0 = (t0 + scale * MLP((f - mean) / std)) / w,  w = 1/m_a + 1/m_b.
//
// Inference runs in BF16 on the matrix cores (v_mfma_f32_16x16x16_bf16,
// FP32 accumulation, the tanh form of GELU).  Every layer is computed transposed (hidden x rows),
// so the accumulator tile of one layer is already the B operand of the
// next: no LDS round trip between layers.  Training kernels are FP32
// VALU: a 64-sample workgroup computes forward and backward passes with
// activations in LDS and writes one partial gradient; a second kernel sums
// the partials in a fixed order (deterministic), then Adam updates.
#include "warmstart.hpp"

#include <cmath>
#include <mutex>

namespace ilves_ws {

using namespace ilves_dev;

namespace {

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// GELU for BF16 inference: the tanh form of Hendrycks and Gimpel,
// 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))) = x / (1 + exp(-2 sqrt(2/pi) (x + 0.044715 x^3))),
// one exp2 and one reciprocal.  Its absolute distance from the exact
// x Phi(x) is below 4.8e-4 (largest near |x| = 2.7), under the BF16
// rounding of the activations that follows (half an ulp is 7.8e-3 there);
// training keeps the library erf.  Saturates to 0 and x for large |x|.
__device__ inline float gelu_fast(float x) {
  constexpr float c = -2.0f * 0.79788456080286536f * 1.4426950408889634f;  // -2 sqrt(2/pi) log2(e)
  const float y = x * __builtin_fmaf(0.044715f * c, x * x, c);
  return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(y));
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bfv4 __attribute__((ext_vector_type(4)));

// four floats -> bfloat16, round to nearest even (two packed hardware
// conversions on gfx950)
__device__ inline bf16x4 to_bf16x4(f32x4 v) { return __builtin_bit_cast(bf16x4, __builtin_convertvector(v, bfv4)); }

// ---------------------------------------------------------------------------
// features: two passes over all rows, one thread per row.  A workgroup takes
// one chunk of up to kChunk consecutive rows of one molecule (the chunk list
// is built with the plan), so the rows of all molecules run in parallel
// whatever the molecule sizes.  Pass 1 computes the row's own quantities and
// keeps its old bond vector in the molecule's workspace; pass 2 sums over
// the constraints sharing an atom.

struct RowCtx {
  MolDesc md;
  int32_t k;
};

template <typename Idx>
__device__ inline RowCtx row_ctx(const DevPlan& P, const int2* __restrict__ chunks) {
  const int2 ch = chunks[blockIdx.x];
  RowCtx c;
  c.md = P.mol[__builtin_amdgcn_readfirstlane(ch.x)];
  c.k = __builtin_amdgcn_readfirstlane(ch.y) + static_cast<int32_t>(threadIdx.x);
  return c;
}

template <typename Idx>
__global__ void __launch_bounds__(kChunk) features_own_kernel(const DevPlan P, const int2* __restrict__ chunks,
                                                            const double* __restrict__ r,
                                                            const double* __restrict__ ru,
                                                            const double* __restrict__ mass, int32_t S,
                                                            unsigned char* __restrict__ ws, float* __restrict__ feat,
                                                            float* __restrict__ wout) {
  const RowCtx c = row_ctx<Idx>(P, chunks);
  const MolDesc& md = c.md;
  const int32_t k = c.k, n = md.n;
  if (k >= n) return;
  const int32_t* inc_ptr = P.inc_ptr + md.incp_off;
  const int64_t R0 = md.row_off;
  double4* er = reinterpret_cast<double4*>(ws + md.ws_off);
  // input atoms (plan-time copies) and local atoms (for the valences) are independent loads
  const int32_t ga = P.ga[R0 + k], gb = P.gb[R0 + k];
  const int32_t la = P.ra[R0 + k], lb = P.rb[R0 + k];
  const double d2 = P.d2[R0 + k];
  const double e0 = r[ga] - r[gb], e1 = r[S + ga] - r[S + gb], e2 = r[2 * S + ga] - r[2 * S + gb];
  const double u0 = ru[ga] - ru[gb], u1 = ru[S + ga] - ru[S + gb], u2 = ru[2 * S + ga] - ru[2 * S + gb];
  const double ia = 1.0 / mass[ga], ib = 1.0 / mass[gb];
  const double w = ia + ib;
  const double ee = e0 * e0 + e1 * e1 + e2 * e2;
  const double bb = u0 * e0 + u1 * e1 + u2 * e2;
  const double cc = u0 * u0 + u1 * u1 + u2 * u2 - d2;
  const double disc = bb * bb - ee * cc;
  // t0 = w * (the decoupled start): the root nearest 0 of |u - t e|^2 = d^2
  // when u.e > 0 and a real root exists, else the Newton step from 0
  const double t0 = (bb > 0.0 && disc >= 0.0) ? cc / (bb + sqrt(disc)) : (bb != 0.0 ? cc / (2.0 * bb) : 0.0);
  const double cx = u1 * e2 - u2 * e1, cy = u2 * e0 - u0 * e2, cz = u0 * e1 - u1 * e0;
  const int32_t dega = inc_ptr[la + 1] - inc_ptr[la], degb = inc_ptr[lb + 1] - inc_ptr[lb];
  float4* f = reinterpret_cast<float4*>(feat + (R0 + k) * N_FEAT);
  f[0] = make_float4(static_cast<float>(t0), static_cast<float>(cc / (2.0 * d2)),
                     static_cast<float>(bb / d2 - 1.0), static_cast<float>(sqrt(cx * cx + cy * cy + cz * cz) / d2));
  f[1] = make_float4(static_cast<float>(fabs(ia - ib) / w), static_cast<float>((dega + degb - 2) * 0.25),
                     static_cast<float>(abs(dega - degb) * 0.25), 0.0f);
  wout[R0 + k] = static_cast<float>(w);
  // the row's old bond vector and w, one 32-byte record for the second pass
  er[k] = make_double4(e0, e1, e2, w);
}

template <typename Idx>
__global__ void __launch_bounds__(kChunk) features_sum_kernel(const DevPlan P, const int2* __restrict__ chunks,
                                                            const double* __restrict__ mass, int32_t S,
                                                            const unsigned char* __restrict__ ws,
                                                            float* __restrict__ feat) {
  const RowCtx c = row_ctx<Idx>(P, chunks);
  const MolDesc& md = c.md;
  const int32_t k = c.k, n = md.n;
  if (k >= n) return;
  (void)S;
  const Layout Lo = struct_layout(n, md.n_levels, md.n_up, md.n_l, md.n_pl, md.n_upd, static_cast<int>(sizeof(Idx)));
  const unsigned char* st = P.ix + md.ix_off;
  const Idx* up_start = reinterpret_cast<const Idx*>(st + Lo.up_start);
  const Idx* l_start = reinterpret_cast<const Idx*>(st + Lo.l_start);
  const Idx* ucol = reinterpret_cast<const Idx*>(st + Lo.ucol);
  // lower-slot records {column, transpose}, indexed by F index t
  const Idx* lpair = reinterpret_cast<const Idx*>(st + Lo.lpair) - 2 * static_cast<int64_t>(md.n_up);
  // per slot: (input index of the shared atom << 1) | (sign < 0), -1 for fill
  const int32_t* gcoef = P.gcoef + md.coef_off;
  const int64_t R0 = md.row_off;
  const double4* er = reinterpret_cast<const double4*>(ws + md.ws_off);
  const double4 ek = er[k];
  const double e0 = ek.x, e1 = ek.y, e2 = ek.z, wk = ek.w;
  const double ee = e0 * e0 + e1 * e1 + e2 * e2;
  double s7 = 0, s8 = 0, s9 = 0, s10 = 0, s11 = 0, s12 = 0, s14 = 0, s15 = 0, cnt = 0;
  // the row's neighbours: its upper slots, then its lower slots, four at a
  // time with all their loads issued before the sums (same summation order)
  const int32_t q0 = up_start[k], nu = up_start[k + 1] - q0;
  const int32_t t0 = l_start[k], tot = nu + (l_start[k + 1] - t0);
  for (int32_t b = 0; b < tot; b += 4) {
    int32_t cf[4], jj[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int32_t idx = b + i;
      const int32_t slot = idx < nu ? q0 + idx : t0 + (idx - nu);
      const bool ok = idx < tot;
      jj[i] = !ok ? k : (idx < nu ? static_cast<int32_t>(ucol[slot]) : static_cast<int32_t>(lpair[2 * slot]));
      cf[i] = ok ? gcoef[slot] : -1;
    }
    double4 ej[4];
    float4 fj[4];
    double mj[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ej[i] = er[jj[i]];
      fj[i] = *reinterpret_cast<const float4*>(feat + (R0 + jj[i]) * N_FEAT);
      mj[i] = mass[cf[i] < 0 ? 0 : cf[i] >> 1];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (cf[i] < 0) continue;  // fill entry or past the row's last slot
      const double sg = (cf[i] & 1) ? -1.0 : 1.0;
      const double fx = ej[i].x, fy = ej[i].y, fz = ej[i].z;
      const double dot = e0 * fx + e1 * fy + e2 * fz;
      const double rho = sg * dot / (mj[i] * wk * ee);
      const double q = wk / ej[i].w;
      s7 += rho * q * fj[i].x;
      s8 += fabs(rho);
      s9 = fmax(s9, fabs(rho));
      s10 += rho * q * fj[i].y;
      s11 += rho * rho;
      s12 += sg * dot / sqrt(ee * (fx * fx + fy * fy + fz * fz));
      s14 += rho * q * fj[i].z;
      s15 += rho * q * fj[i].w;
      cnt += 1.0;
    }
  }
  float* f = feat + (R0 + k) * N_FEAT;
  f[7] = static_cast<float>(s7);
  reinterpret_cast<float4*>(f)[2] = make_float4(static_cast<float>(s8), static_cast<float>(s9),
                                                static_cast<float>(s10), static_cast<float>(s11));
  reinterpret_cast<float4*>(f)[3] = make_float4(static_cast<float>(s12 / fmax(cnt, 1.0)),
                                                static_cast<float>(cnt / 6.0), static_cast<float>(s14),
                                                static_cast<float>(s15));
}

// ---------------------------------------------------------------------------
// BF16 MFMA inference.  Tile = 16 rows per wave.  Operand layouts of
// v_mfma_f32_16x16x16_bf16 (lane l, i = 0..3):
//   A (16 x 16, M x K): A[l % 16][4 (l / 16) + i]
//   B (16 x 16, K x N): B[4 (l / 16) + i][l % 16]
//   C (16 x 16):        C[4 (l / 16) + i][l % 16]
// Layers are computed transposed, H^T = W^T X^T: A = W^T blocks, B = the
// transposed activations (K = features or hidden units, N = rows).

__global__ void __launch_bounds__(256) mlp_infer_kernel(const float* __restrict__ params,
                                                        const float* __restrict__ norm,
                                                        const float* __restrict__ feat, const float* __restrict__ w,
                                                        const int32_t* __restrict__ cid, int32_t n_rows,
                                                        double* __restrict__ lambda) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;   // row of the tile (N index)
  const int kq = lane >> 4;    // which group of 4 along K / M
  const float* W1 = params;
  const float* b1 = W1 + N_FEAT * N_HID;
  const float* W2 = b1 + N_HID;
  const float* b2 = W2 + N_HID * N_HID;
  const float* W3 = b2 + N_HID;
  const float b3 = W3[N_HID];
  const float* mean = norm;
  const float* sdev = norm + N_FEAT;
  const float scale = norm[2 * N_FEAT];

  // weights as A operands: A1[hb] = W1^T block, A2[ob][kb] = W2^T block
  bf16x4 A1[4], A2[4][4];
  float bias1[4][4], bias2[4][4], w3[4][4];
#pragma unroll
  for (int hb = 0; hb < 4; ++hb) {
    f32x4 a;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = W1[(4 * kq + i) * N_HID + 16 * hb + col];
      bias1[hb][i] = b1[16 * hb + 4 * kq + i];
      bias2[hb][i] = b2[16 * hb + 4 * kq + i];
      w3[hb][i] = W3[16 * hb + 4 * kq + i];
    }
    A1[hb] = to_bf16x4(a);
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob)
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      f32x4 a;
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = W2[(16 * kb + 4 * kq + i) * N_HID + 16 * ob + col];
      A2[ob][kb] = to_bf16x4(a);
    }
  // this lane's four features are normalised as (f - mean) * (1 / std)
  f32x4 fmean, finv;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    fmean[i] = mean[4 * kq + i];
    finv[i] = 1.0f / sdev[4 * kq + i];
  }

  const int n_tiles = (n_rows + 15) / 16;
  for (int tile = blockIdx.x * 4 + wave; tile < n_tiles; tile += gridDim.x * 4) {
    const int row = tile * 16 + col;
    const bool valid = row < n_rows;
    f32x4 x = {0.0f, 0.0f, 0.0f, 0.0f};
    if (valid) {
      x = *reinterpret_cast<const f32x4*>(feat + static_cast<int64_t>(row) * N_FEAT + 4 * kq);
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = (x[i] - fmean[i]) * finv[i];
    }
    const bf16x4 xb = to_bf16x4(x);
    bf16x4 h1[4];
#pragma unroll
    for (int hb = 0; hb < 4; ++hb) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A1[hb], xb, acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = gelu_fast(acc[i] + bias1[hb][i]);
      h1[hb] = to_bf16x4(acc);
    }
    float part = 0.0f;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A2[ob][kb], h1[kb], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) part += w3[ob][i] * gelu_fast(acc[i] + bias2[ob][i]);
    }
    // lanes l, l+16, l+32, l+48 hold partial sums of the same row
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (kq == 0 && valid) {
      const float o = part + b3;
      const float t = feat[static_cast<int64_t>(row) * N_FEAT] + scale * o;
      lambda[cid[row]] = static_cast<double>(t) / static_cast<double>(w[row]);
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 training kernels

__global__ void __launch_bounds__(256) mlp_block_kernel(const float* __restrict__ params,
                                                        const float* __restrict__ x, const float* __restrict__ y,
                                                        int32_t n, float inv_n, float* __restrict__ part,
                                                        float* __restrict__ out, int grad) {
  __shared__ float X[TRAIN_BS][N_FEAT];
  __shared__ float Z1[TRAIN_BS][N_HID + 1];
  __shared__ float H1[TRAIN_BS][N_HID + 1];
  __shared__ float Z2[TRAIN_BS][N_HID + 1];
  __shared__ float H2[TRAIN_BS][N_HID + 1];
  __shared__ float dO[TRAIN_BS];
  __shared__ float sq[TRAIN_BS];
  const int tid = threadIdx.x;
  const float* W1 = params;
  const float* b1 = W1 + N_FEAT * N_HID;
  const float* W2 = b1 + N_HID;
  const float* b2 = W2 + N_HID * N_HID;
  const float* W3 = b2 + N_HID;
  const float b3 = W3[N_HID];
  const int64_t s0 = static_cast<int64_t>(blockIdx.x) * TRAIN_BS;
  const int nb = static_cast<int>(min<int64_t>(TRAIN_BS, n - s0));

  for (int e = tid; e < TRAIN_BS * N_FEAT; e += 256) {
    const int s = e / N_FEAT, f = e % N_FEAT;
    X[s][f] = s < nb ? x[(s0 + s) * N_FEAT + f] : 0.0f;
  }
  __syncthreads();
  for (int e = tid; e < TRAIN_BS * N_HID; e += 256) {
    const int s = e / N_HID, h = e % N_HID;
    float z = b1[h];
    for (int f = 0; f < N_FEAT; ++f) z += X[s][f] * W1[f * N_HID + h];
    Z1[s][h] = z;
    H1[s][h] = gelu(z);
  }
  __syncthreads();
  for (int e = tid; e < TRAIN_BS * N_HID; e += 256) {
    const int s = e / N_HID, h = e % N_HID;
    float z = b2[h];
    for (int i = 0; i < N_HID; ++i) z += H1[s][i] * W2[i * N_HID + h];
    Z2[s][h] = z;
    H2[s][h] = gelu(z);
  }
  __syncthreads();
  if (tid < TRAIN_BS) {
    const int s = tid;
    float o = b3;
    for (int h = 0; h < N_HID; ++h) o += H2[s][h] * W3[h];
    if (!grad) {
      if (s < nb) out[s0 + s] = o;
    } else {
      const float r = s < nb ? o - y[s0 + s] : 0.0f;
      dO[s] = r * inv_n;
      sq[s] = 0.5f * r * r * inv_n;
    }
  }
  if (!grad) return;
  __syncthreads();
  for (int e = tid; e < TRAIN_BS * N_HID; e += 256) {  // dZ2 into Z2
    const int s = e / N_HID, h = e % N_HID;
    Z2[s][h] = dO[s] * W3[h] * gelu_grad(Z2[s][h]);
  }
  __syncthreads();
  for (int e = tid; e < TRAIN_BS * N_HID; e += 256) {  // dZ1 into Z1
    const int s = e / N_HID, i = e % N_HID;
    float acc = 0.0f;
    for (int h = 0; h < N_HID; ++h) acc += Z2[s][h] * W2[i * N_HID + h];
    Z1[s][i] = acc * gelu_grad(Z1[s][i]);
  }
  __syncthreads();
  float* g = part + static_cast<int64_t>(blockIdx.x) * (N_PARAMS + 1);
  for (int p = tid; p <= N_PARAMS; p += 256) {
    float acc = 0.0f;
    int q = p;
    if (q < N_FEAT * N_HID) {
      const int f = q / N_HID, h = q % N_HID;
      for (int s = 0; s < TRAIN_BS; ++s) acc += X[s][f] * Z1[s][h];
    } else if ((q -= N_FEAT * N_HID) < N_HID) {
      for (int s = 0; s < TRAIN_BS; ++s) acc += Z1[s][q];
    } else if ((q -= N_HID) < N_HID * N_HID) {
      const int i = q / N_HID, h = q % N_HID;
      for (int s = 0; s < TRAIN_BS; ++s) acc += H1[s][i] * Z2[s][h];
    } else if ((q -= N_HID * N_HID) < N_HID) {
      for (int s = 0; s < TRAIN_BS; ++s) acc += Z2[s][q];
    } else if ((q -= N_HID) < N_HID) {
      for (int s = 0; s < TRAIN_BS; ++s) acc += dO[s] * H2[s][q];
    } else if ((q -= N_HID) < 1) {
      for (int s = 0; s < TRAIN_BS; ++s) acc += dO[s];
    } else {
      for (int s = 0; s < TRAIN_BS; ++s) acc += sq[s];  // loss
    }
    g[p] = acc;
  }
}

__global__ void reduce_partials(const float* __restrict__ part, int32_t nblocks, float* __restrict__ grad,
                                float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > N_PARAMS) return;
  float acc = 0.0f;
  for (int b = 0; b < nblocks; ++b) acc += part[static_cast<int64_t>(b) * (N_PARAMS + 1) + p];
  if (p < N_PARAMS) grad[p] = acc;
  else *loss = acc;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int32_t n, float lr, float beta1, float beta2, float eps,
                            float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

}  // namespace

hipError_t launch_features(const DevPlan& P, const int2* chunks, int32_t n_chunks, bool wide, const double* r,
                           const double* r_u, const double* mass, int32_t n_atoms, unsigned char* ws, float* feat,
                           float* w, hipStream_t stream) {
  (void)hipGetLastError();  // no stale error from an earlier call
  if (n_chunks <= 0) return hipSuccess;
  if (wide) {
    hipLaunchKernelGGL(features_own_kernel<int32_t>, dim3(n_chunks), dim3(kChunk), 0, stream, P, chunks, r, r_u,
                       mass, n_atoms, ws, feat, w);
    hipLaunchKernelGGL(features_sum_kernel<int32_t>, dim3(n_chunks), dim3(kChunk), 0, stream, P, chunks, mass,
                       n_atoms, ws, feat);
  } else {
    hipLaunchKernelGGL(features_own_kernel<uint16_t>, dim3(n_chunks), dim3(kChunk), 0, stream, P, chunks, r, r_u,
                       mass, n_atoms, ws, feat, w);
    hipLaunchKernelGGL(features_sum_kernel<uint16_t>, dim3(n_chunks), dim3(kChunk), 0, stream, P, chunks, mass,
                       n_atoms, ws, feat);
  }
  return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* params, const float* norm, const float* feat, const float* w,
                            const int32_t* cid, int32_t n_rows, double* lambda, hipStream_t stream) {
  (void)hipGetLastError();  // no stale error from an earlier call
  if (n_rows <= 0) return hipSuccess;
  const int tiles = (n_rows + 15) / 16;
  const int blocks = (tiles + 3) / 4 < 2048 ? (tiles + 3) / 4 : 2048;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(blocks), dim3(256), 0, stream, params, norm, feat, w, cid, n_rows,
                     lambda);
  return hipGetLastError();
}

hipError_t launch_mlp_forward_f32(const float* params, const float* x, int32_t n, float* out, hipStream_t stream) {
  (void)hipGetLastError();  // no stale error from an earlier call
  if (n <= 0) return hipSuccess;
  const int blocks = (n + TRAIN_BS - 1) / TRAIN_BS;
  hipLaunchKernelGGL(mlp_block_kernel, dim3(blocks), dim3(256), 0, stream, params, x, nullptr, n, 0.0f, nullptr,
                     out, 0);
  return hipGetLastError();
}

hipError_t launch_mlp_grad_f32(const float* params, const float* x, const float* y, int32_t n, float* grad,
                               float* loss, float* work, hipStream_t stream) {
  (void)hipGetLastError();  // no stale error from an earlier call
  if (n <= 0) return hipErrorInvalidValue;
  const int blocks = (n + TRAIN_BS - 1) / TRAIN_BS;
  hipLaunchKernelGGL(mlp_block_kernel, dim3(blocks), dim3(256), 0, stream, params, x, y, n, 1.0f / n, work,
                     nullptr, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partials, dim3((N_PARAMS + 1 + 255) / 256), dim3(256), 0, stream, work, blocks, grad,
                     loss);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gradient without a caller workspace, for callers that cannot allocate
// (HIP graph capture, tight training loops): the per-workgroup partial
// gradients go to this file-scope device array.  Each GPU holds its own copy
// of it (until the process ends).  In host code the name `scratch` is only a
// host-side stand-in, never a device address: the address is looked up once
// per device with hipGetSymbolAddress, with that device current, and that
// pointer is what the kernels receive.  Every call overwrites the partials
// it reads (ceil(n / TRAIN_BS) whole records), so nothing has to start at
// zero; two calls that overlap on one GPU race on the array.
static __device__ __align__(256) float scratch[kStaticGradBlocks * (N_PARAMS + 1)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_grad_scratch(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_mlp_grad_f32_static(const float* params, const float* x, const float* y, int32_t n, float* grad,
                                      float* loss, hipStream_t stream) {
  if (n <= 0 || n > kStaticGradBlocks * TRAIN_BS) return hipErrorInvalidValue;
  float* work = nullptr;
  const hipError_t e = static_grad_scratch(&work);
  if (e != hipSuccess) return e;
  return launch_mlp_grad_f32(params, x, y, n, grad, loss, work, stream);
}

hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t n, float lr, float beta1,
                           float beta2, float eps, int32_t step, hipStream_t stream) {
  (void)hipGetLastError();  // no stale error from an earlier call
  if (n <= 0 || step < 1) return hipErrorInvalidValue;
  const float bc1 = 1.0f - powf(beta1, static_cast<float>(step));
  const float bc2 = 1.0f - powf(beta2, static_cast<float>(step));
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, params, grad, m, v, n, lr, beta1,
                     beta2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace ilves_ws
