// Measurement of one design choice (gfx950): the predictor's spatial
// derivative contraction on the matrix cores against the vector ALUs.
//
// In the space-time predictor (eq. CGfinal) each element needs, at every time
// node of every Picard sweep, d/dxi and d/deta of its ten exchanged fields (q,
// the flux components and the node coordinates): D_xi and D_eta (nb x nb, nb =
// 6 at M = 2) applied to a 6 x 10 block. The step's kernel (k_predict) keeps
// one lane per spatial node and takes the element's other nodes from LDS, so
// each lane forms 20 dot products of length 6. Here the same contraction, in
// the same lane layout and the same LDS exchange, is run either that way or
// with v_mfma_f64_16x16x4f64 over the wavefront's ten elements (A = [D_xi;
// D_eta] padded to 16 x 8, B = the exchanged fields, 100 columns in 7 tiles of
// 16, two k-steps each), the results handed back to the node lanes through
// LDS. The fields are fed back (q <- q/2 + (d_xi + d_eta)/20) for `iters`
// rounds so that the data stay on chip and both variants do the same dependent
// work. Not part of the step: the library measures with it (ader_probe_contraction).
#include <hip/hip_runtime.h>

#include "aderweno.h"
#include "common.h"

namespace aw {
namespace {

constexpr int TPB = 256;
constexpr int PM = 2;                       // the order measured
constexpr int NB = (PM + 1) * (PM + 2) / 2; // 6 spatial nodes
constexpr int NFLD = 10;
constexpr int EPW = 64 / NB;                // 10 elements per wavefront, 4 spare lanes
constexpr int WPB = TPB / 64;
constexpr int COLS = EPW * NFLD;            // 100 (element, field) columns per wavefront
constexpr int TILES = (COLS + 15) / 16;     // 7

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline void probe_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// F and out: [n][NFLD][NB] (element, field, node).
template <bool MFMA>
__global__ void __launch_bounds__(TPB) k_probe_contract(const Tables* __restrict__ tb, int n, int iters,
                                                        const double* __restrict__ F, double* __restrict__ out) {
  __shared__ double ex[WPB][EPW + 1][NFLD][NB];      // exchanged fields (slot EPW: spare lanes)
  __shared__ double res[MFMA ? WPB : 1][EPW][NFLD][12];
  const int wv = threadIdx.x / 64, lw = threadIdx.x % 64;
  const bool spare = lw >= EPW * NB;
  const int el = spare ? EPW : lw / NB;
  const int m = spare ? lw - EPW * NB : lw % NB;
  double Dx[NB], De[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    Dx[k] = tb->Dxi[m][k];
    De[k] = tb->Deta[m][k];
  }
  // MFMA A operand: lane l holds A[l % 16][l / 16 + 4 s] for k-step s
  double a0 = 0.0, a1 = 0.0;
  if (MFMA) {
    const int i = lw % 16, k0 = lw / 16, k1 = 4 + lw / 16;
    auto A = [&](int r, int k) {
      if (k >= NB) return 0.0;
      return r < NB ? tb->Dxi[r][k] : (r < 2 * NB ? tb->Deta[r - NB][k] : 0.0);
    };
    a0 = A(i, k0);
    a1 = A(i, k1);
  }
  for (int base = (blockIdx.x * WPB + wv) * EPW; base < n; base += gridDim.x * WPB * EPW) {
    const int e = base + el;
    const bool live = !spare && e < n;
    double q[NFLD];
#pragma unroll
    for (int f = 0; f < NFLD; ++f) q[f] = live ? F[(size_t(e) * NFLD + f) * NB + m] : 1.0;
#pragma unroll 1
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int f = 0; f < NFLD; ++f) ex[wv][el][f][m] = q[f];
      probe_wave_sync();
      double r[NFLD];
      if (!MFMA) {
#pragma unroll
        for (int f = 0; f < NFLD; ++f) {
          double da = 0.0, db = 0.0;
#pragma unroll
          for (int k = 0; k < NB; ++k) {
            da += Dx[k] * ex[wv][el][f][k];
            db += De[k] * ex[wv][el][f][k];
          }
          r[f] = da + db;
        }
      } else {
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
          const int col = lw % 16 + 16 * t;
          const bool valid = col < COLS;
          const int ce = valid ? col / NFLD : 0, cf = valid ? col % NFLD : 0;
          const int k0 = lw / 16, k1 = 4 + lw / 16;
          const double b0 = valid ? ex[wv][ce][cf][k0] : 0.0;
          const double b1 = valid && k1 < NB ? ex[wv][ce][cf][k1] : 0.0;
          d4 acc = {0.0, 0.0, 0.0, 0.0};
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc, 0, 0, 0);
          // D[i][j] sits in lane j + 16 (i % 4), register i / 4
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int row = lw / 16 + 4 * g;
            if (valid && row < 2 * NB) res[wv][ce][cf][row] = acc[g];
          }
        }
        probe_wave_sync();
#pragma unroll
        for (int f = 0; f < NFLD; ++f) r[f] = spare ? 0.0 : res[wv][el][f][m] + res[wv][el][f][NB + m];
      }
      probe_wave_sync();
#pragma unroll
      for (int f = 0; f < NFLD; ++f) q[f] = 0.5 * q[f] + 0.05 * r[f];
    }
    if (live) {
#pragma unroll
      for (int f = 0; f < NFLD; ++f) out[(size_t(e) * NFLD + f) * NB + m] = q[f];
    }
  }
}

}  // namespace

int probe_contraction(const Tables* tab, int use_mfma, long n, int iters, const double* F, double* out,
                      void* stream, int blocks) {
  if (blocks <= 0) {
    long b = (n + WPB * EPW - 1) / (WPB * EPW);
    blocks = int(b > 16384 ? 16384 : (b < 1 ? 1 : b));
  }
  if (use_mfma)
    hipLaunchKernelGGL((k_probe_contract<true>), dim3(blocks), dim3(TPB), 0, (hipStream_t)stream, tab, int(n), iters,
                       F, out);
  else
    hipLaunchKernelGGL((k_probe_contract<false>), dim3(blocks), dim3(TPB), 0, (hipStream_t)stream, tab, int(n),
                       iters, F, out);
  return int(hipGetLastError());
}

}  // namespace aw
