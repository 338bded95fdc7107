// Learned list size: a small network proposes each cell's k from local
// density features; the security-radius certificate still judges every cell,
// so results do not depend on the network.
//
//  * k_features   12 features per query from its 16-NN list and the grid.
//  * k_mlp        BF16 MFMA (v_mfma_f32_16x16x16bf16_1k, FP32 accumulate)
//                 forward pass for 16-sample tiles; in training mode also
//                 softmax cross-entropy and the backward pass, accumulating
//                 per-block weight gradients with MFMA (sum over samples
//                 as the K dimension).  Inference writes the chosen bucket.
//  * k_reduce     deterministic fixed-order sum of the per-block partials.
//  * k_adam       Adam on FP32 master weights.
//
// MFMA operand layout (16x16x16, wave64, lane l, element i = 0..3):
//   A[m][k]: m = l % 16, k = 4 (l / 16) + i;   B[k][n]: k = 4 (l / 16) + i, n = l % 16
//   D[m][n]: m = 4 (l / 16) + i, n = l % 16
// so a product's D registers are, unchanged, the A operand of its transpose
// and the B operand of a product over the same rows; the other hand-offs go
// through LDS.
#include "internal.h"
#include "device_common.h"

#include <cfloat>
#include <climits>
#include <cmath>
#include <cstring>

namespace votess {
constexpr int NF = VOTESS_NFEAT, NH = VOTESS_NHID, NO = VOTESS_NBUCKET;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH, NPARAM = OFF_B3 + NO;
static_assert(NPARAM == VOTESS_NPARAM, "parameter layout");
constexpr int kSamplesPerBlock = 64;  // four 16-sample tiles per wave
__device__ constexpr int kBuckets[VOTESS_NBUCKET] = {8, 12, 16, 24, 32, 48, 64};
}  // namespace votess

struct votess_kmodel {
  votess_ctx* ctx = nullptr;
  float* theta = nullptr;  // [NPARAM] FP32 master weights
  float* m = nullptr;      // Adam moments
  float* v = nullptr;
  float* norm = nullptr;   // [24]: mean[12], std[12]
  float* grads = nullptr;  // [NPARAM]
  float* partial = nullptr;
  int partial_blocks = 0;
  int step = 0;
};

namespace votess {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float((unsigned)bf16_bits(f) << 16); }
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 r;
  r[0] = (short)bf16_bits(a);
  r[1] = (short)bf16_bits(b);
  r[2] = (short)bf16_bits(c);
  r[3] = (short)bf16_bits(d);
  return r;
}
__device__ __forceinline__ floatx4 mfma(bf16x4 a, bf16x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// --------------------------------------------------------------- features
// Closed-form eigenvalues of a symmetric 3x3 matrix, largest first.
__device__ void eig3(double a00, double a01, double a02, double a11, double a12, double a22, double e[3]) {
  const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const double q = (a00 + a11 + a22) / 3.0;
  const double p2 = (a00 - q) * (a00 - q) + (a11 - q) * (a11 - q) + (a22 - q) * (a22 - q) + 2.0 * p1;
  if (!(p2 > 0.0)) {
    e[0] = e[1] = e[2] = q;
    return;
  }
  const double p = sqrt(p2 / 6.0);
  const double b00 = (a00 - q) / p, b11 = (a11 - q) / p, b22 = (a22 - q) / p;
  const double b01 = a01 / p, b02 = a02 / p, b12 = a12 / p;
  const double det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02);
  const double r = fmin(1.0, fmax(-1.0, 0.5 * det));
  const double phi = acos(r) / 3.0;
  e[0] = q + 2.0 * p * cos(phi);
  e[2] = q + 2.0 * p * cos(phi + 2.0943951023931954923);
  e[1] = 3.0 * q - e[0] - e[2];
}

template <typename T>
__global__ __launch_bounds__(256) void k_features(const typename Rec<T>::type* __restrict__ rec, int n, GridDev G,
                                                  const int* __restrict__ cell_start, const int* __restrict__ queries,
                                                  int nq, const int* __restrict__ knn16, int kstride,
                                                  float* __restrict__ feats) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int s = queries ? queries[q] : q;
  const auto pr = rec[s];
  const double px = pr.x, py = pr.y, pz = pr.z;
  const int cx = axis_cell(px, G.lo0, G.ih0, G.g0), cy = axis_cell(py, G.lo1, G.ih1, G.g1),
            cz = axis_cell(pz, G.lo2, G.ih2, G.g2);
  const double ncells = (double)G.g0 * G.g1 * G.g2;
  const double nbar = (double)n / ncells;
  const double vol = (G.hi0 - G.lo0) * (G.hi1 - G.lo1) * (G.hi2 - G.lo2);
  const double ell = cbrt(vol / (double)n);
  float f[NF];
  for (int sc = 0; sc < 3; ++sc) {
    const int x0 = max(cx - sc, 0), x1 = min(cx + sc, G.g0 - 1);
    const int y0 = max(cy - sc, 0), y1 = min(cy + sc, G.g1 - 1);
    const int z0 = max(cz - sc, 0), z1 = min(cz + sc, G.g2 - 1);
    long long cnt = 0;
    for (int z = z0; z <= z1; ++z)
      for (int y = y0; y <= y1; ++y) {
        const int row = G.g0 * (y + G.g1 * z);
        cnt += cell_start[row + x1 + 1] - cell_start[row + x0];
      }
    const double c = (double)(x1 - x0 + 1) * (y1 - y0 + 1) * (z1 - z0 + 1);
    f[sc] = (float)log2(1.0 + (double)cnt / (nbar * c));
  }
  const int* L = knn16 + (size_t)q * kstride;  // the row's first 16 entries
  double d[16], ox[16], oy[16], oz[16];
  int m = 0;
  for (int i = 0; i < 16; ++i) {
    const int j = L[i];
    if (j < 0) break;
    const auto qr = rec[j];
    ox[m] = (double)qr.x - px;
    oy[m] = (double)qr.y - py;
    oz[m] = (double)qr.z - pz;
    d[m] = sqrt(ox[m] * ox[m] + oy[m] * oy[m] + oz[m] * oz[m]);
    ++m;
  }
  if (m == 0) {
    for (int i = 3; i < NF; ++i) f[i] = 0.0f;
  } else {
    auto dk = [&](int k) { return d[min(k, m) - 1]; };
    f[3] = (float)log2(dk(4) / ell);
    f[4] = (float)log2(dk(8) / ell);
    f[5] = (float)log2(dk(16) / ell);
    double mx = 0, my = 0, mz = 0;
    for (int i = 0; i < m; ++i) {
      mx += ox[i];
      my += oy[i];
      mz += oz[i];
    }
    mx /= m;
    my /= m;
    mz /= m;
    f[6] = (float)(sqrt(mx * mx + my * my + mz * mz) / dk(16));
    f[7] = (float)log2(dk(1) / ell);
    double c00 = 0, c01 = 0, c02 = 0, c11 = 0, c12 = 0, c22 = 0;
    for (int i = 0; i < m; ++i) {
      const double a = ox[i] - mx, b = oy[i] - my, c = oz[i] - mz;
      c00 += a * a; c01 += a * b; c02 += a * c; c11 += b * b; c12 += b * c; c22 += c * c;
    }
    double e[3];
    eig3(c00 / m, c01 / m, c02 / m, c11 / m, c12 / m, c22 / m, e);
    const double tr = e[0] + e[1] + e[2];
    for (int i = 0; i < 3; ++i) f[8 + i] = tr > 0 ? (float)(e[i] / tr) : (float)(1.0 / 3.0);
    const double wall = fmin(fmin(fmin(px - G.lo0, G.hi0 - px), fmin(py - G.lo1, G.hi1 - py)),
                             fmin(pz - G.lo2, G.hi2 - pz));
    f[11] = (float)fmin(wall / dk(16), 4.0);
  }
  for (int i = 0; i < NF; ++i) feats[(size_t)q * NF + i] = f[i];
}

// ------------------------------------------------------------------ network
struct MlpArgs {
  const float* theta;
  const float* norm;
  const float* feats;
  const uint8_t* labels;
  int nb;
  float inv_batch;
  float tau;
  float* partial;   // train: [blocks][NPARAM + 1] (last: loss sum)
  uint8_t* bucket;  // choose: [nb]
  float* logits;    // forward: [nb][NO] (nullable)
};

// mode 0: forward (logits and / or bucket), 1: forward + backward partials
template <int MODE>
__global__ __launch_bounds__(64) void k_mlp(MlpArgs a) {
  const int l = threadIdx.x;
  const int r = l & 15, g4 = l >> 4;  // A/B: row / column r, k-group g4; D: row 4 g4 + i, column r
  __shared__ unsigned short hs[16 * NH];  // activations / signals in [sample][unit] (bf16 bits)
  __shared__ float ps[16 * 16];           // logits -> probabilities [sample][output]
  const float* th = a.theta;
  // weights as bf16 operands
  bf16x4 W1B[4], W2B[4][4], W3B[4], W3T[4], W2T[4][4];
  for (int nt = 0; nt < 4; ++nt) {  // layer 1: B[k=f][n=u] = W1[u][f]
    float w[4];
    for (int i = 0; i < 4; ++i) {
      const int f = 4 * g4 + i;
      w[i] = f < NF ? th[OFF_W1 + (16 * nt + r) * NF + f] : 0.0f;
    }
    W1B[nt] = pack4(w[0], w[1], w[2], w[3]);
  }
  for (int kt = 0; kt < 4; ++kt)
    for (int nt = 0; nt < 4; ++nt) {  // layer 2: B[k=u1][n=u2] = W2[u2][u1]
      float w[4], wt[4];
      for (int i = 0; i < 4; ++i) {
        w[i] = th[OFF_W2 + (16 * nt + r) * NH + 16 * kt + 4 * g4 + i];
        wt[i] = th[OFF_W2 + (16 * kt + 4 * g4 + i) * NH + 16 * nt + r];  // backward: B[k=u2][n=u1] = W2[u2][u1]
      }
      W2B[kt][nt] = pack4(w[0], w[1], w[2], w[3]);
      W2T[kt][nt] = pack4(wt[0], wt[1], wt[2], wt[3]);
    }
  for (int kt = 0; kt < 4; ++kt) {  // layer 3: B[k=u][n=o] = W3[o][u]
    float w[4];
    for (int i = 0; i < 4; ++i) w[i] = r < NO ? th[OFF_W3 + r * NH + 16 * kt + 4 * g4 + i] : 0.0f;
    W3B[kt] = pack4(w[0], w[1], w[2], w[3]);
  }
  for (int nt = 0; nt < 4; ++nt) {  // backward: B[k=o][n=u] = W3[o][u]
    float w[4];
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * g4 + i;
      w[i] = o < NO ? th[OFF_W3 + o * NH + 16 * nt + r] : 0.0f;
    }
    W3T[nt] = pack4(w[0], w[1], w[2], w[3]);
  }
  float b1[4], b2[4];
  for (int nt = 0; nt < 4; ++nt) {
    b1[nt] = th[OFF_B1 + 16 * nt + r];
    b2[nt] = th[OFF_B2 + 16 * nt + r];
  }
  const float b3 = r < NO ? th[OFF_B3 + r] : 0.0f;
  float mean[4], sdv[4];
  for (int i = 0; i < 4; ++i) {
    const int f = 4 * g4 + i;
    mean[i] = f < NF ? a.norm[f] : 0.0f;
    sdv[i] = f < NF ? a.norm[NF + f] : 1.0f;
  }

  // backward accumulators (D layout)
  floatx4 gW1[4], gW2[4][4], gW3[4];
  const floatx4 z4 = {0.f, 0.f, 0.f, 0.f};
  for (int t = 0; t < 4; ++t) {
    gW1[t] = z4;
    gW3[t] = z4;
    for (int u = 0; u < 4; ++u) gW2[t][u] = z4;
  }
  float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gb3 = 0.0f, loss = 0.0f;

  const int tiles_total = (a.nb + 15) / 16;
  // training: block b owns tiles 4b..4b+3 (its partial sums are per block);
  // inference: grid-stride over tiles
  const int t_begin = MODE == 1 ? blockIdx.x * 4 : blockIdx.x;
  const int t_end = MODE == 1 ? min(tiles_total, blockIdx.x * 4 + 4) : tiles_total;
  const int t_step = MODE == 1 ? 1 : gridDim.x;
  for (int tile = t_begin; tile < t_end; tile += t_step) {
    {
      const int base = tile * 16;
      // ---- inputs: A layout X[s=r][f=4 g4 + i]
      float xa[4];
      const int sa = base + r;
      for (int i = 0; i < 4; ++i) {
        const int f = 4 * g4 + i;
        const float v = (sa < a.nb && f < NF) ? a.feats[(size_t)sa * NF + f] : 0.0f;
        xa[i] = (f < NF && sa < a.nb) ? bf16_round((v - mean[i]) / sdv[i]) : 0.0f;
      }
      const bf16x4 XA = pack4(xa[0], xa[1], xa[2], xa[3]);
      // ---- layer 1
      floatx4 z1[4];
      bf16x4 H1D[4];
      for (int nt = 0; nt < 4; ++nt) {
        z1[nt] = mfma(XA, W1B[nt], z4);
        float h[4];
        for (int i = 0; i < 4; ++i) {
          z1[nt][i] += b1[nt];
          h[i] = bf16_round(fmaxf(z1[nt][i], 0.0f));
          hs[(4 * g4 + i) * NH + 16 * nt + r] = bf16_bits(h[i]);
        }
        H1D[nt] = pack4(h[0], h[1], h[2], h[3]);
      }
      __syncthreads();
      bf16x4 H1A[4];
      for (int kt = 0; kt < 4; ++kt) {
        bf16x4 v;
        for (int i = 0; i < 4; ++i) v[i] = (short)hs[r * NH + 16 * kt + 4 * g4 + i];
        H1A[kt] = v;
      }
      __syncthreads();
      // ---- layer 2
      floatx4 z2[4];
      bf16x4 H2D[4];
      for (int nt = 0; nt < 4; ++nt) {
        floatx4 acc = z4;
        for (int kt = 0; kt < 4; ++kt) acc = mfma(H1A[kt], W2B[kt][nt], acc);
        float h[4];
        for (int i = 0; i < 4; ++i) {
          acc[i] += b2[nt];
          h[i] = bf16_round(fmaxf(acc[i], 0.0f));
          hs[(4 * g4 + i) * NH + 16 * nt + r] = bf16_bits(h[i]);
        }
        z2[nt] = acc;
        H2D[nt] = pack4(h[0], h[1], h[2], h[3]);
      }
      __syncthreads();
      bf16x4 H2A[4];
      for (int kt = 0; kt < 4; ++kt) {
        bf16x4 v;
        for (int i = 0; i < 4; ++i) v[i] = (short)hs[r * NH + 16 * kt + 4 * g4 + i];
        H2A[kt] = v;
      }
      // ---- layer 3: logits D[s = 4 g4 + i][o = r]
      floatx4 z3 = z4;
      for (int kt = 0; kt < 4; ++kt) z3 = mfma(H2A[kt], W3B[kt], z3);
      for (int i = 0; i < 4; ++i) ps[(4 * g4 + i) * 16 + r] = z3[i] + b3;
      __syncthreads();
      // ---- softmax per sample (lanes 0..15, one sample each)
      if (l < 16) {
        const int s = base + l;
        float mx = -FLT_MAX;
        for (int o = 0; o < NO; ++o) mx = fmaxf(mx, ps[l * 16 + o]);
        float e[NO], sum = 0.0f;
        for (int o = 0; o < NO; ++o) {
          e[o] = expf(ps[l * 16 + o] - mx);
          sum += e[o];
        }
        if (MODE == 0 && s < a.nb) {
          if (a.logits)
            for (int o = 0; o < NO; ++o) a.logits[(size_t)s * NO + o] = ps[l * 16 + o];
          if (a.bucket) {
            float c = 0.0f;
            int b = NO - 1;
            for (int o = 0; o < NO - 1; ++o) {
              c += e[o];
              if (c >= a.tau * sum) {
                b = o;
                break;
              }
            }
            a.bucket[s] = (uint8_t)b;
          }
        }
        if (MODE == 1) {
          const int y = s < a.nb ? a.labels[s] : 0;
          if (s < a.nb) loss += ((mx + logf(sum)) - ps[l * 16 + y]) * a.inv_batch;
          for (int o = 0; o < 16; ++o) {
            float g = 0.0f;
            if (o < NO && s < a.nb) g = (e[o] / sum - (o == y ? 1.0f : 0.0f)) * a.inv_batch;
            ps[l * 16 + o] = g;
          }
        }
      }
      __syncthreads();
      if (MODE == 1) {
        // ---- G3 in D layout [s = 4 g4 + i][o = r]; db3; dW3 += G3^T H2
        float g3[4];
        for (int i = 0; i < 4; ++i) g3[i] = ps[(4 * g4 + i) * 16 + r];
        gb3 += g3[0] + g3[1] + g3[2] + g3[3];
        const bf16x4 G3D = pack4(g3[0], g3[1], g3[2], g3[3]);
        for (int nt = 0; nt < 4; ++nt) gW3[nt] = mfma(G3D, H2D[nt], gW3[nt]);
        // G3 in A layout [s = r][o = 4 g4 + i] (rounded)
        bf16x4 G3A;
        for (int i = 0; i < 4; ++i) G3A[i] = (short)bf16_bits(ps[r * 16 + 4 * g4 + i]);
        // ---- dH2 = G3 W3, G2 = dH2 * (z2 > 0)
        float g2[4][4];
        for (int nt = 0; nt < 4; ++nt) {
          const floatx4 dh = mfma(G3A, W3T[nt], z4);
          for (int i = 0; i < 4; ++i) {
            g2[nt][i] = z2[nt][i] > 0.0f ? dh[i] : 0.0f;
            gb2[nt] += g2[nt][i];
          }
        }
        __syncthreads();
        bf16x4 G2D[4];
        for (int nt = 0; nt < 4; ++nt) {
          G2D[nt] = pack4(g2[nt][0], g2[nt][1], g2[nt][2], g2[nt][3]);
          for (int i = 0; i < 4; ++i) hs[(4 * g4 + i) * NH + 16 * nt + r] = bf16_bits(g2[nt][i]);
        }
        // dW2[u2][u1] += G2^T H1
        for (int mt = 0; mt < 4; ++mt)
          for (int nt = 0; nt < 4; ++nt) gW2[mt][nt] = mfma(G2D[mt], H1D[nt], gW2[mt][nt]);
        __syncthreads();
        bf16x4 G2A[4];
        for (int kt = 0; kt < 4; ++kt) {
          bf16x4 v;
          for (int i = 0; i < 4; ++i) v[i] = (short)hs[r * NH + 16 * kt + 4 * g4 + i];
          G2A[kt] = v;
        }
        // ---- dH1 = G2 W2, G1 = dH1 * (z1 > 0); dW1 += G1^T X
        bf16x4 XB;  // B layout X[s = 4 g4 + i][f = r]
        {
          float xb[4];
          for (int i = 0; i < 4; ++i) {
            const int s = base + 4 * g4 + i;
            const float v = (s < a.nb && r < NF) ? a.feats[(size_t)s * NF + r] : 0.0f;
            xb[i] = (s < a.nb && r < NF) ? bf16_round((v - a.norm[r]) / a.norm[NF + r]) : 0.0f;
          }
          XB = pack4(xb[0], xb[1], xb[2], xb[3]);
        }
        for (int nt = 0; nt < 4; ++nt) {
          floatx4 dh = z4;
          for (int kt = 0; kt < 4; ++kt) dh = mfma(G2A[kt], W2T[kt][nt], dh);
          float g1[4];
          for (int i = 0; i < 4; ++i) {
            g1[i] = z1[nt][i] > 0.0f ? dh[i] : 0.0f;
            gb1[nt] += g1[i];
          }
          gW1[nt] = mfma(pack4(g1[0], g1[1], g1[2], g1[3]), XB, gW1[nt]);
        }
        __syncthreads();
      }
    }
  }
  if (MODE == 1) {
    float* out = a.partial + (size_t)blockIdx.x * (NPARAM + 1);
    // weights: D layout rows 4 g4 + i, column r
    for (int mt = 0; mt < 4; ++mt)
      for (int i = 0; i < 4; ++i) {
        const int u = 16 * mt + 4 * g4 + i;
        if (r < NF) out[OFF_W1 + u * NF + r] = gW1[mt][i];
        for (int nt = 0; nt < 4; ++nt) out[OFF_W2 + u * NH + 16 * nt + r] = gW2[mt][nt][i];
      }
    for (int nt = 0; nt < 4; ++nt)
      for (int i = 0; i < 4; ++i) {
        const int o = 4 * g4 + i;
        if (o < NO) out[OFF_W3 + o * NH + 16 * nt + r] = gW3[nt][i];
      }
    // biases: reduce over the four row groups
    for (int nt = 0; nt < 4; ++nt) {
      float v1 = gb1[nt], v2 = gb2[nt];
      v1 += __shfl_xor(v1, 16, 64);
      v1 += __shfl_xor(v1, 32, 64);
      v2 += __shfl_xor(v2, 16, 64);
      v2 += __shfl_xor(v2, 32, 64);
      if (g4 == 0) {
        out[OFF_B1 + 16 * nt + r] = v1;
        out[OFF_B2 + 16 * nt + r] = v2;
      }
    }
    float v3 = gb3;
    v3 += __shfl_xor(v3, 16, 64);
    v3 += __shfl_xor(v3, 32, 64);
    if (g4 == 0 && r < NO) out[OFF_B3 + r] = v3;
    float ls = loss;
    for (int o = 1; o < 64; o <<= 1) ls += __shfl_xor(ls, o, 64);
    if (l == 0) out[NPARAM] = ls;
  }
}


// Fixed-order sum of per-block partials: grads[p] = sum_b partial[b][p].
__global__ void k_reduce(const float* __restrict__ partial, int blocks, float* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > NPARAM) return;
  float acc = 0.0f;
  for (int b = 0; b < blocks; ++b) acc += partial[(size_t)b * (NPARAM + 1) + p];
  out[p] = acc;
}

__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float gi = g[p];
  const float mi = 0.9f * m[p] + 0.1f * gi;
  const float vi = 0.999f * v[p] + 0.001f * gi * gi;
  m[p] = mi;
  v[p] = vi;
  theta[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// Training label of a cell from the method's own run (status and k_needed of
// the label-recording clip): the least bucket b with buckets[b] >= k_needed,
// or the largest bucket when the cell was not certified by its list or
// needed more than the largest bucket.
__global__ void k_labels(const uint8_t* __restrict__ status, const int* __restrict__ kneeded, int n,
                         uint8_t* __restrict__ labels) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int kn = status[i] == VOTESS_CELL_CERTIFIED ? kneeded[i] : INT_MAX;
  int b = 0;
  while (b < NO - 1 && kBuckets[b] < kn) ++b;
  labels[i] = (uint8_t)b;
}

// Standardisation statistics, deterministic: each block sums x and x^2 of
// every feature in double over a fixed strided range (a fixed-order tree in
// LDS), then one block adds the partials in block order.
constexpr int kNormBlocks = 256;
__global__ __launch_bounds__(256) void k_norm_partial(const float* __restrict__ feats, int n,
                                                      double* __restrict__ partial) {
  __shared__ double red[256];
  for (int f = 0; f < 2 * NF; ++f) {
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
      const double x = feats[(size_t)i * NF + (f % NF)];
      acc += f < NF ? x : x * x;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * 2 * NF + f] = red[0];
    __syncthreads();
  }
}

// mean = S1 / n, std = sqrt(max(S2 / n - mean^2, 0)) + 1e-6 (population std)
__global__ void k_norm_final(const double* __restrict__ partial, int blocks, int n, float* __restrict__ norm) {
  const int f = threadIdx.x;
  if (f >= NF) return;
  double s1 = 0.0, s2 = 0.0;
  for (int b = 0; b < blocks; ++b) {
    s1 += partial[(size_t)b * 2 * NF + f];
    s2 += partial[(size_t)b * 2 * NF + NF + f];
  }
  const double mean = s1 / n;
  const double var = fmax(s2 / n - mean * mean, 0.0);
  norm[f] = (float)mean;
  norm[NF + f] = (float)(sqrt(var) + 1e-6);
}

}  // namespace

votess_status run_features(votess_ctx* ctx, const void* sorted, votess_dtype dt, int n, const GridDev& G,
                           const int32_t* cell_start, const SubGrid& sub, const int32_t* queries, int nq,
                           int32_t* knn16, float* feats, hipStream_t st) {
  if (nq == 0) return VOTESS_OK;
  VT_TRY(launch_knn(ctx, sorted, dt, n, G, cell_start, sub, queries, nq, 16,
                    dt == VOTESS_F32 ? VOTESS_F32 : VOTESS_F64, knn16, st));
  const unsigned b = (unsigned)((nq + 255) / 256);
  if (dt == VOTESS_F32)
    k_features<float><<<b, 256, 0, st>>>((const float4*)sorted, n, G, cell_start, queries, nq, knn16, 16, feats);
  else
    k_features<double><<<b, 256, 0, st>>>((const double4*)sorted, n, G, cell_start, queries, nq, knn16, 16, feats);
  VT_HIP(hipGetLastError());
  return VOTESS_OK;
}

votess_status run_choose(votess_kmodel* km, const float* feats, int nq, float tau, uint8_t* bucket, float* logits,
                         hipStream_t st) {
  if (nq == 0) return VOTESS_OK;
  MlpArgs a{};
  a.theta = km->theta;
  a.norm = km->norm;
  a.feats = feats;
  a.nb = nq;
  a.tau = tau;
  a.bucket = bucket;
  a.logits = logits;
  const int tiles = (nq + 15) / 16;
  const int blocks = std::max(1, std::min(tiles, 256 * 16));
  k_mlp<0><<<blocks, 64, 0, st>>>(a);
  VT_HIP(hipGetLastError());
  return VOTESS_OK;
}

static votess_status run_grad(votess_kmodel* km, const float* feats, const uint8_t* labels, int nb, hipStream_t st) {
  const int blocks = (nb + kSamplesPerBlock - 1) / kSamplesPerBlock;
  if (blocks > km->partial_blocks) {
    dev_free(km->ctx, km->partial);
    km->partial = (float*)dev_alloc(km->ctx, (size_t)blocks * (NPARAM + 1) * sizeof(float));
    if (!km->partial) return fail(VOTESS_ENOMEM, "kmodel partial gradients");
    km->partial_blocks = blocks;
  }
  MlpArgs a{};
  a.theta = km->theta;
  a.norm = km->norm;
  a.feats = feats;
  a.labels = labels;
  a.nb = nb;
  a.inv_batch = 1.0f / (float)nb;
  a.partial = km->partial;
  k_mlp<1><<<blocks, 64, 0, st>>>(a);
  VT_HIP(hipGetLastError());
  k_reduce<<<(NPARAM + 1 + 255) / 256, 256, 0, st>>>(km->partial, blocks, km->grads);
  VT_HIP(hipGetLastError());
  return VOTESS_OK;
}

// Learned first pass of votess_tessellate: one k-NN pass at the largest
// bucket for every cell, the features from each row's first 16 entries, the
// network's bucket per cell, then per bucket a clip pass over the first k
// entries of its cells' rows; with `stream` the clip pass goes on by grid
// rings where the list does not certify (else those cells are left for the
// retry ladder).
votess_status learned_first_pass(votess_ctx* ctx, votess_kmodel* km, double tau, const void* sorted, int n,
                                 const votess_grid& grid, const int32_t* cell_start, const ClipLaunch& base,
                                 int stream, int32_t* cells_buf, votess_stats& S, hipStream_t st) {
  // The k-NN runs once, at the largest bucket, for every cell: a row is
  // sorted by (d^2, sorted index), so its first 16 entries are the cell's
  // 16-NN list (the features' input) and its first k entries the k-list of
  // a cell the network puts in bucket k.  A separate 16-NN pass would cost
  // about a third of this one, more than the shorter lists of the smaller
  // buckets save.
  const GridDev G = to_dev(grid);
  const votess_dtype dist = base.knn_dist;
  const int KL = votess_buckets[NO - 1];
  void* knn = dev_alloc(ctx, (size_t)n * KL * 4);
  void* feats = dev_alloc(ctx, (size_t)n * NF * 4);
  void* bucket = dev_alloc(ctx, (size_t)n);
  void* failbuf = dev_alloc(ctx, (size_t)n * 4);
  auto cleanup = [&]() {
    dev_free(ctx, knn);
    dev_free(ctx, feats);
    dev_free(ctx, bucket);
    dev_free(ctx, failbuf);
  };
  if (!knn || !feats || !bucket || !failbuf) {
    cleanup();
    return fail(VOTESS_ENOMEM, "learned pass buffers");
  }
  hipEvent_t e0, e1, e2, e3;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventCreate(&e2);
  (void)hipEventCreate(&e3);
  (void)hipEventRecord(e0, st);
  votess_status rc =
      launch_knn(ctx, sorted, base.dtype, n, G, cell_start, base.sub, nullptr, n, KL, dist, (int32_t*)knn, st);
  (void)hipEventRecord(e1, st);
  if (rc == VOTESS_OK && n > 0) {
    const unsigned b = (unsigned)((n + 255) / 256);
    if (base.dtype == VOTESS_F32)
      k_features<float><<<b, 256, 0, st>>>((const float4*)sorted, n, G, cell_start, nullptr, n, (const int*)knn, KL,
                                           (float*)feats);
    else
      k_features<double><<<b, 256, 0, st>>>((const double4*)sorted, n, G, cell_start, nullptr, n, (const int*)knn,
                                            KL, (float*)feats);
    if (hipGetLastError() != hipSuccess) rc = fail(VOTESS_EHIP, "learned pass: feature kernel launch");
  }
  (void)hipEventRecord(e2, st);
  if (rc == VOTESS_OK) rc = run_choose(km, (const float*)feats, n, (float)tau, (uint8_t*)bucket, nullptr, st);
  (void)hipEventRecord(e3, st);
  (void)hipEventSynchronize(e3);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  S.ms_knn += ms;
  (void)hipEventElapsedTime(&ms, e1, e2);
  S.ms_features += ms;
  (void)hipEventElapsedTime(&ms, e2, e3);
  S.ms_mlp += ms;
  int64_t entered_prev = 0;
  if (base.counters) {
    unsigned long long e = 0;
    if (hipMemcpyAsync(&e, base.counters + 5, 8, hipMemcpyDeviceToHost, st) == hipSuccess &&
        hipStreamSynchronize(st) == hipSuccess)
      entered_prev = (int64_t)e;
  }
  for (int b = 0; b < NO && rc == VOTESS_OK; ++b) {
    int cnt = 0;
    // the compaction takes a status mask; bucket values are 0..6, so bit b selects bucket b
    rc = launch_compact_failed((const uint8_t*)bucket, nullptr, n, cells_buf, ctx->d_counter,
                               (uint8_t)(1u << b), ctx->ws, st);
    if (rc != VOTESS_OK) break;
    if (hipMemcpyAsync(&cnt, ctx->d_counter, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(VOTESS_EHIP, "learned pass: bucket count");
      break;
    }
    S.bucket_cells[b] = cnt;
    if (cnt == 0) continue;
    const int k = votess_buckets[b];
    (void)hipEventRecord(e0, st);
    ClipLaunch c = base;
    c.cells = cells_buf;
    c.nc = cnt;
    c.knn = (const int32_t*)knn;
    c.k = k;
    c.knn_stride = KL;
    c.knn_by_id = 1;
    c.stream = stream;
    rc = launch_clip(c, st);
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(&ms, e0, e1);
    S.ms_clip += ms;
    if (rc != VOTESS_OK) break;
    // cells of this bucket still uncertified after the pass, and cells its
    // lists left uncertified that went on into the stream phase
    int nfail = 0;
    unsigned long long entered = 0;
    rc = launch_compact_failed(base.status, cells_buf, cnt, (int32_t*)failbuf, ctx->d_counter,
                               (uint8_t)((1u << VOTESS_CELL_RADIUS) | (1u << VOTESS_CELL_CAPACITY)), ctx->ws, st);
    if (rc != VOTESS_OK) break;
    if (hipMemcpyAsync(&nfail, ctx->d_counter, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        (base.counters && hipMemcpyAsync(&entered, base.counters + 5, 8, hipMemcpyDeviceToHost, st) != hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(VOTESS_EHIP, "learned pass: failure count");
      break;
    }
    if (S.npasses < VOTESS_MAX_PASSES) {
      S.pass_k[S.npasses] = k;
      S.pass_cells[S.npasses] = cnt;
      S.pass_failed[S.npasses] = nfail;
      S.pass_streamed[S.npasses] = (int64_t)entered - entered_prev;
      S.npasses++;
    }
    entered_prev = (int64_t)entered;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  (void)hipEventDestroy(e3);
  cleanup();
  return rc;
}

}  // namespace votess

// ------------------------------------------- allocation-free feature pass
// Scratch of votess_features_noalloc: the 16-NN lists of at most
// kNoAllocMaxQ queries (4 MiB), held by every device the library runs on
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host it is only a stand-in for the symbol): the device
// address is looked up once per context (votess_create, with the context's
// device current) and kept in ctx->noalloc_scratch.
constexpr int64_t kNoAllocMaxQ = 65536;
static __device__ __align__(256) int32_t scratch[kNoAllocMaxQ * 16];

namespace votess {
votess_status init_noalloc_scratch(votess_ctx* ctx) {
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(VOTESS_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  ctx->noalloc_scratch = p;
  return VOTESS_OK;
}
}  // namespace votess

// ------------------------------------------------------------------ C ABI
using namespace votess;

namespace {
uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
}  // namespace

extern "C" {

votess_kmodel* votess_kmodel_create(votess_ctx* ctx, uint64_t seed) {
  if (!ctx) {
    fail(VOTESS_EINVAL, "kmodel_create: null ctx");
    return nullptr;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    fail(VOTESS_EHIP, "kmodel_create: hipSetDevice");
    return nullptr;
  }
  votess_kmodel* km = new votess_kmodel;
  km->ctx = ctx;
  km->theta = (float*)dev_alloc(ctx, NPARAM * 4);
  km->m = (float*)dev_alloc(ctx, NPARAM * 4);
  km->v = (float*)dev_alloc(ctx, NPARAM * 4);
  km->norm = (float*)dev_alloc(ctx, 2 * NF * 4);
  km->grads = (float*)dev_alloc(ctx, (NPARAM + 1) * 4);
  if (!km->theta || !km->m || !km->v || !km->norm || !km->grads) {
    votess_kmodel_destroy(km);
    fail(VOTESS_ENOMEM, "kmodel_create");
    return nullptr;
  }
  // He-uniform weights, zero biases, identity standardisation
  std::vector<float> th(NPARAM, 0.0f), nm(2 * NF, 0.0f);
  uint64_t st = seed;
  auto uni = [&](float lim) { return lim * (2.0f * (float)((splitmix(st) >> 11) * (1.0 / 9007199254740992.0)) - 1.0f); };
  for (int i = 0; i < NH * NF; ++i) th[OFF_W1 + i] = uni(std::sqrt(6.0f / NF));
  for (int i = 0; i < NH * NH; ++i) th[OFF_W2 + i] = uni(std::sqrt(6.0f / NH));
  for (int i = 0; i < NO * NH; ++i) th[OFF_W3 + i] = uni(std::sqrt(6.0f / NH));
  for (int f = 0; f < NF; ++f) nm[NF + f] = 1.0f;
  if (hipMemcpy(km->theta, th.data(), NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(km->norm, nm.data(), 2 * NF * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(km->m, 0, NPARAM * 4) != hipSuccess || hipMemset(km->v, 0, NPARAM * 4) != hipSuccess) {
    votess_kmodel_destroy(km);
    fail(VOTESS_EHIP, "kmodel_create: upload");
    return nullptr;
  }
  return km;
}

void votess_kmodel_destroy(votess_kmodel* km) {
  if (!km) return;
  votess_ctx* ctx = km->ctx;
  dev_free(ctx, km->theta);
  dev_free(ctx, km->m);
  dev_free(ctx, km->v);
  dev_free(ctx, km->norm);
  dev_free(ctx, km->grads);
  dev_free(ctx, km->partial);
  delete km;
}

votess_status votess_kmodel_set_params(votess_kmodel* km, const float* params_h, const float* mean_h,
                                       const float* std_h) {
  if (!km) return fail(VOTESS_EINVAL, "kmodel is null");
  VT_HIP(hipSetDevice(km->ctx->device));
  if (params_h) {
    VT_HIP(hipMemcpy(km->theta, params_h, NPARAM * 4, hipMemcpyHostToDevice));
    VT_HIP(hipMemset(km->m, 0, NPARAM * 4));
    VT_HIP(hipMemset(km->v, 0, NPARAM * 4));
    km->step = 0;
  }
  if (mean_h) VT_HIP(hipMemcpy(km->norm, mean_h, NF * 4, hipMemcpyHostToDevice));
  if (std_h) {
    for (int f = 0; f < NF; ++f)
      if (!(std_h[f] > 0.0f)) return fail(VOTESS_EINVAL, "kmodel: std must be positive");
    VT_HIP(hipMemcpy(km->norm + NF, std_h, NF * 4, hipMemcpyHostToDevice));
  }
  return VOTESS_OK;
}

votess_status votess_kmodel_get_params(votess_kmodel* km, float* params_h, float* mean_h, float* std_h) {
  if (!km) return fail(VOTESS_EINVAL, "kmodel is null");
  VT_HIP(hipSetDevice(km->ctx->device));
  VT_HIP(hipDeviceSynchronize());
  if (params_h) VT_HIP(hipMemcpy(params_h, km->theta, NPARAM * 4, hipMemcpyDeviceToHost));
  if (mean_h) VT_HIP(hipMemcpy(mean_h, km->norm, NF * 4, hipMemcpyDeviceToHost));
  if (std_h) VT_HIP(hipMemcpy(std_h, km->norm + NF, NF * 4, hipMemcpyDeviceToHost));
  return VOTESS_OK;
}

votess_status votess_features(votess_ctx* ctx, const void* sorted, int64_t n, const votess_grid* grid,
                              const int32_t* cell_start, const int32_t* subinfo, const int32_t* sub_start,
                              const int32_t* queries, int64_t nq, float* feats, void* stream) {
  if (!ctx || !grid) return fail(VOTESS_EINVAL, "features: null ctx/grid");
  if (!queries) nq = n;
  if (n < 1 || nq < 0 || n >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "features: bad sizes");
  if (nq > 0 && (!sorted || !cell_start || !feats)) return fail(VOTESS_EINVAL, "features: null buffer");
  VT_TRY(check_sub(subinfo, sub_start, n, "features"));
  VT_HIP(hipSetDevice(ctx->device));
  void* knn16 = dev_alloc(ctx, (size_t)std::max<int64_t>(nq, 1) * 16 * 4);
  if (!knn16) return fail(VOTESS_ENOMEM, "features: 16-NN buffer");
  hipStream_t st = (hipStream_t)stream;
  SubGrid sg;
  sg.info = (const int2*)subinfo;
  sg.start = sub_start;
  votess_status rc = run_features(ctx, sorted, VOTESS_F32, (int)n, to_dev(*grid), cell_start, sg, queries, (int)nq,
                                  (int32_t*)knn16, feats, st);
  (void)hipStreamSynchronize(st);
  dev_free(ctx, knn16);
  return rc;
}

int64_t votess_features_noalloc_max(void) { return kNoAllocMaxQ; }

votess_status votess_features_noalloc(votess_ctx* ctx, const void* sorted, int64_t n, const votess_grid* grid,
                                      const int32_t* cell_start, const int32_t* subinfo, const int32_t* sub_start,
                                      const int32_t* queries, int64_t nq, float* feats, void* stream) {
  if (!ctx || !grid) return fail(VOTESS_EINVAL, "features_noalloc: null ctx/grid");
  if (!queries) nq = n;
  if (n < 1 || nq < 0 || n >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "features_noalloc: bad sizes");
  if (nq > kNoAllocMaxQ)
    return fail(VOTESS_EINVAL, "features_noalloc: %lld queries exceed the static scratch (at most %lld)",
                (long long)nq, (long long)kNoAllocMaxQ);
  if (nq > 0 && (!sorted || !cell_start || !feats)) return fail(VOTESS_EINVAL, "features_noalloc: null buffer");
  VT_TRY(check_sub(subinfo, sub_start, n, "features_noalloc"));
  if (!ctx->noalloc_scratch) return fail(VOTESS_EHIP, "features_noalloc: scratch address not set up");
  VT_HIP(hipSetDevice(ctx->device));
  SubGrid sg;
  sg.info = (const int2*)subinfo;
  sg.start = sub_start;
  return run_features(ctx, sorted, VOTESS_F32, (int)n, to_dev(*grid), cell_start, sg, queries, (int)nq,
                      (int32_t*)ctx->noalloc_scratch, feats, (hipStream_t)stream);
}

votess_status votess_kmodel_forward(votess_kmodel* km, const float* feats, int64_t nq, float* logits, void* stream) {
  if (!km || (nq > 0 && (!feats || !logits))) return fail(VOTESS_EINVAL, "kmodel_forward: null argument");
  if (nq < 0 || nq >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "kmodel_forward: bad size");
  VT_HIP(hipSetDevice(km->ctx->device));
  return run_choose(km, feats, (int)nq, 1.0f, nullptr, logits, (hipStream_t)stream);
}

votess_status votess_kmodel_choose(votess_kmodel* km, const float* feats, int64_t nq, float tau, uint8_t* bucket,
                                   void* stream) {
  if (!km || (nq > 0 && (!feats || !bucket))) return fail(VOTESS_EINVAL, "kmodel_choose: null argument");
  if (nq < 0 || nq >= (1LL << 31) - 1 || !(tau > 0.0f && tau <= 1.0f))
    return fail(VOTESS_EINVAL, "kmodel_choose: bad size or tau");
  VT_HIP(hipSetDevice(km->ctx->device));
  return run_choose(km, feats, (int)nq, tau, bucket, nullptr, (hipStream_t)stream);
}

votess_status votess_kmodel_grad(votess_kmodel* km, const float* feats, const uint8_t* labels, int64_t nb,
                                 float* grads, float* loss, void* stream) {
  if (!km || !feats || !labels || !grads || !loss) return fail(VOTESS_EINVAL, "kmodel_grad: null argument");
  if (nb < 1 || nb >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "kmodel_grad: bad batch");
  VT_HIP(hipSetDevice(km->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  VT_TRY(run_grad(km, feats, labels, (int)nb, st));
  VT_HIP(hipMemcpyAsync(grads, km->grads, NPARAM * 4, hipMemcpyDeviceToDevice, st));
  VT_HIP(hipMemcpyAsync(loss, km->grads + NPARAM, 4, hipMemcpyDeviceToDevice, st));
  return VOTESS_OK;
}

votess_status votess_kmodel_train_step(votess_kmodel* km, const float* feats, const uint8_t* labels, int64_t nb,
                                       float lr, float* loss, void* stream) {
  if (!km || !feats || !labels) return fail(VOTESS_EINVAL, "kmodel_train_step: null argument");
  if (nb < 1 || nb >= (1LL << 31) - 1 || !(lr > 0.0f)) return fail(VOTESS_EINVAL, "kmodel_train_step: bad batch/lr");
  VT_HIP(hipSetDevice(km->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  VT_TRY(run_grad(km, feats, labels, (int)nb, st));
  km->step += 1;
  const float c1 = 1.0f - std::pow(0.9f, (float)km->step), c2 = 1.0f - std::pow(0.999f, (float)km->step);
  k_adam<<<(NPARAM + 255) / 256, 256, 0, st>>>(km->theta, km->m, km->v, km->grads, lr, c1, c2);
  VT_HIP(hipGetLastError());
  if (loss) VT_HIP(hipMemcpyAsync(loss, km->grads + NPARAM, 4, hipMemcpyDeviceToDevice, st));
  return VOTESS_OK;
}


/* ---- versioned blob: the weights, the standardisation and tau ---------- */
namespace {
constexpr uint32_t kBlobMagic = 0x4D4B5456u;  // "VTKM"
constexpr uint32_t kBlobVersion = 1;
struct BlobHead {
  uint32_t magic, version, nfeat, nhid, nbucket, nparam;
  int32_t buckets[VOTESS_NBUCKET];
  uint32_t pad;
  double tau;
};
constexpr size_t kBlobBytes = sizeof(BlobHead) + (size_t)(NPARAM + 2 * NF) * 4 + 8;
uint64_t fnv1a(const unsigned char* p, size_t len) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < len; ++i) h = (h ^ p[i]) * 0x100000001b3ull;
  return h;
}
}  // namespace

size_t votess_kmodel_blob_size(void) { return kBlobBytes; }

votess_status votess_kmodel_save(votess_kmodel* km, double tau, void* blob_h, size_t cap, size_t* len_h) {
  if (!km) return fail(VOTESS_EINVAL, "kmodel_save: null model");
  if (len_h) *len_h = kBlobBytes;
  if (!blob_h) return VOTESS_OK;
  if (cap < kBlobBytes) return fail(VOTESS_ECAPACITY, "kmodel_save: blob needs %zu bytes, got %zu", kBlobBytes, cap);
  if (!(tau > 0.0 && tau <= 1.0)) return fail(VOTESS_EINVAL, "kmodel_save: tau must be in (0, 1]");
  std::vector<unsigned char> buf(kBlobBytes, 0);
  BlobHead h{};
  h.magic = kBlobMagic;
  h.version = kBlobVersion;
  h.nfeat = NF;
  h.nhid = NH;
  h.nbucket = NO;
  h.nparam = NPARAM;
  for (int b = 0; b < NO; ++b) h.buckets[b] = votess_buckets[b];
  h.tau = tau;
  std::memcpy(buf.data(), &h, sizeof(h));
  float* body = (float*)(buf.data() + sizeof(h));
  VT_TRY(votess_kmodel_get_params(km, body, body + NPARAM, body + NPARAM + NF));
  const uint64_t sum = fnv1a(buf.data(), kBlobBytes - 8);
  std::memcpy(buf.data() + kBlobBytes - 8, &sum, 8);
  std::memcpy(blob_h, buf.data(), kBlobBytes);
  return VOTESS_OK;
}

votess_status votess_kmodel_load(votess_ctx* ctx, const void* blob_h, size_t len, votess_kmodel** out_h,
                                 double* tau_h) {
  if (!ctx || !blob_h || !out_h) return fail(VOTESS_EINVAL, "kmodel_load: null argument");
  *out_h = nullptr;
  if (len != kBlobBytes) return fail(VOTESS_EINVAL, "kmodel_load: blob of %zu bytes, expected %zu", len, kBlobBytes);
  const unsigned char* b = (const unsigned char*)blob_h;
  BlobHead h;
  std::memcpy(&h, b, sizeof(h));
  if (h.magic != kBlobMagic) return fail(VOTESS_EINVAL, "kmodel_load: not a k-model blob");
  if (h.version != kBlobVersion) return fail(VOTESS_EINVAL, "kmodel_load: blob version %u, expected %u", h.version, kBlobVersion);
  if (h.nfeat != (uint32_t)NF || h.nhid != (uint32_t)NH || h.nbucket != (uint32_t)NO || h.nparam != (uint32_t)NPARAM)
    return fail(VOTESS_EINVAL, "kmodel_load: network shape differs from this library's");
  for (int i = 0; i < NO; ++i)
    if (h.buckets[i] != votess_buckets[i]) return fail(VOTESS_EINVAL, "kmodel_load: bucket sizes differ");
  uint64_t sum;
  std::memcpy(&sum, b + kBlobBytes - 8, 8);
  if (sum != fnv1a(b, kBlobBytes - 8)) return fail(VOTESS_EINVAL, "kmodel_load: checksum mismatch");
  if (!(h.tau > 0.0 && h.tau <= 1.0)) return fail(VOTESS_EINVAL, "kmodel_load: bad tau");
  std::vector<float> body(NPARAM + 2 * NF);
  std::memcpy(body.data(), b + sizeof(h), body.size() * 4);
  votess_kmodel* km = votess_kmodel_create(ctx, 0);
  if (!km) return VOTESS_ENOMEM;
  const votess_status rc = votess_kmodel_set_params(km, body.data(), body.data() + NPARAM, body.data() + NPARAM + NF);
  if (rc != VOTESS_OK) {
    votess_kmodel_destroy(km);
    return rc;
  }
  *out_h = km;
  if (tau_h) *tau_h = h.tau;
  return VOTESS_OK;
}

votess_status votess_kmodel_labels(votess_ctx* ctx, const uint8_t* status, const int32_t* kneeded, int64_t n,
                                   uint8_t* labels, void* stream) {
  if (!ctx) return fail(VOTESS_EINVAL, "kmodel_labels: null ctx");
  if (n < 0 || n >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "kmodel_labels: bad size");
  if (n > 0 && (!status || !kneeded || !labels)) return fail(VOTESS_EINVAL, "kmodel_labels: null buffer");
  if (n == 0) return VOTESS_OK;
  VT_HIP(hipSetDevice(ctx->device));
  k_labels<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(status, kneeded, (int)n, labels);
  VT_HIP(hipGetLastError());
  return VOTESS_OK;
}

votess_status votess_kmodel_fit_norm(votess_kmodel* km, const float* feats, int64_t n, void* stream) {
  if (!km) return fail(VOTESS_EINVAL, "kmodel_fit_norm: null model");
  if (n < 1 || n >= (1LL << 31) - 1 || !feats) return fail(VOTESS_EINVAL, "kmodel_fit_norm: bad features");
  VT_HIP(hipSetDevice(km->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)std::min<int64_t>(kNormBlocks, (n + 255) / 256);
  double* partial = (double*)dev_alloc(km->ctx, (size_t)blocks * 2 * NF * sizeof(double));
  if (!partial) return fail(VOTESS_ENOMEM, "kmodel_fit_norm: partial sums");
  k_norm_partial<<<blocks, 256, 0, st>>>(feats, (int)n, partial);
  k_norm_final<<<1, 64, 0, st>>>(partial, blocks, (int)n, km->norm);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamSynchronize(st);
  dev_free(km->ctx, partial);
  if (e1 != hipSuccess || e2 != hipSuccess) return fail(VOTESS_EHIP, "kmodel_fit_norm: kernels failed");
  return VOTESS_OK;
}

}  // extern "C"
