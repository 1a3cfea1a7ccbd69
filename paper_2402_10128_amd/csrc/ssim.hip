// ssim.hip -- SSIM term of the GES training loss (lambda_ssim L_ssim, Sec. 5 loss) and its gradient.
//
// Gaussian-weighted SSIM (Wang et al., 2004): 11x11 window (sigma 1.5, unit sum), each colour channel on its
// own, zero padding so the map has the image's size, C1 = 0.01^2, C2 = 0.03^2; L_ssim = 1 - mean SSIM over
// every pixel and channel.  The gradient goes through the five local statistics: with A, B, Cxy the
// derivatives of SSIM(p) with respect to w*x, w*x^2 and w*xy at p, d(sum_p SSIM)/dx(q) =
// (w*A)(q) + 2 x(q) (w*B)(q) + y(q) (w*Cxy)(q), w symmetric and zero-padded.
//
// Two tiled passes over 32x32 pixel tiles, each staging the tile plus a 5-pixel halo in LDS and filtering
// separably (11 taps across, then 11 down):
//   forward: the five statistics of every channel -> SSIM (summed per block) and the maps A, B, Cxy;
//   backward: the three maps filtered again -> dL/dI, added to the caller's gradient.
// The statistics are taken of x - 1/2 and y - 1/2 (padding becomes -1/2): variances and covariances do not
// change under a common shift, and the second moments of values in [-1/2, 1/2] lose four times less to
// the cancellation in E[x^2] - E[x]^2.  A final block adds the per-block sums in a fixed order.
//
// Memory per pixel and channel: the forward reads x, y (8 B) and writes three maps (12 B); the backward
// reads the maps (12 B), x, y and the gradient (12 B) and writes the gradient (4 B).  Halo re-reads hit L2.
#include <algorithm>
#include <cmath>

#include "ges_internal.h"

namespace ges {

constexpr int kSsimR = 5;
constexpr int kSsimTaps = 2 * kSsimR + 1;
constexpr int kSsimT = 32;                       // output tile edge
constexpr int kSsimIn = kSsimT + 2 * kSsimR;     // staged edge (42)
constexpr int kSsimPitch = kSsimIn + 1;
constexpr int kSsimThreads = 256;
constexpr int kSsimRowsPerThread = kSsimT * kSsimT / kSsimThreads;   // 4 outputs per thread and channel
constexpr float kSsimC1 = 0.01f * 0.01f, kSsimC2 = 0.03f * 0.03f;
constexpr float kSsimShift = 0.5f;

struct SsimWeights {
  float w[kSsimTaps];
};

__global__ void __launch_bounds__(kSsimThreads) ssim_fwd_kernel(const float* __restrict__ img,
                                                                const float* __restrict__ tgt, int w, int h,
                                                                const SsimWeights wt, float* __restrict__ maps,
                                                                double* __restrict__ partial) {
  __shared__ float sx[3][kSsimIn][kSsimPitch];
  __shared__ float sy[3][kSsimIn][kSsimPitch];
  __shared__ float hs[5][kSsimIn][kSsimT];
  __shared__ double red[kSsimThreads / 64];
  const int t = threadIdx.x;
  const int x0 = blockIdx.x * kSsimT - kSsimR, y0 = blockIdx.y * kSsimT - kSsimR;
  // stage both images (all three channels, rows of 42 interleaved pixels = 126 contiguous floats)
  for (int e = t; e < kSsimIn * kSsimIn * 3; e += kSsimThreads) {
    const int r = e / (kSsimIn * 3), j = e - r * (kSsimIn * 3);
    const int col = j / 3, c = j - col * 3;
    const int gx = x0 + col, gy = y0 + r;
    float a = -kSsimShift, b = -kSsimShift;
    if (gx >= 0 && gx < w && gy >= 0 && gy < h) {
      const size_t o = 3 * ((size_t)gy * w + gx) + c;
      a = img[o] - kSsimShift;
      b = tgt[o] - kSsimShift;
    }
    sx[c][r][col] = a;
    sy[c][r][col] = b;
  }
  const size_t plane = (size_t)w * h;
  float ssum = 0.f;
  for (int c = 0; c < 3; ++c) {
    __syncthreads();
    for (int i = t; i < kSsimIn * kSsimT; i += kSsimThreads) {
      const int r = i / kSsimT, col = i - r * kSsimT;
      float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
      for (int k = 0; k < kSsimTaps; ++k) {
        const float a = sx[c][r][col + k], b = sy[c][r][col + k], wk = wt.w[k];
        m0 += wk * a;
        m1 += wk * b;
        m2 += wk * (a * a);
        m3 += wk * (b * b);
        m4 += wk * (a * b);
      }
      hs[0][r][col] = m0;
      hs[1][r][col] = m1;
      hs[2][r][col] = m2;
      hs[3][r][col] = m3;
      hs[4][r][col] = m4;
    }
    __syncthreads();
    const int ox = t % kSsimT;
#pragma unroll
    for (int j = 0; j < kSsimRowsPerThread; ++j) {
      const int oy = t / kSsimT + j * (kSsimThreads / kSsimT);
      float ex = 0.f, ey = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
      for (int k = 0; k < kSsimTaps; ++k) {
        const float wk = wt.w[k];
        ex += wk * hs[0][oy + k][ox];
        ey += wk * hs[1][oy + k][ox];
        exx += wk * hs[2][oy + k][ox];
        eyy += wk * hs[3][oy + k][ox];
        exy += wk * hs[4][oy + k][ox];
      }
      const int gx = x0 + kSsimR + ox, gy = y0 + kSsimR + oy;
      if (gx >= w || gy >= h) continue;
      // shifted moments -> variances/covariance; means of the unshifted images
      const float vx = exx - ex * ex, vy = eyy - ey * ey, cxy = exy - ex * ey;
      const float mx = ex + kSsimShift, my = ey + kSsimShift;
      const float n1 = 2.f * mx * my + kSsimC1, n2 = 2.f * cxy + kSsimC2;
      const float d1 = mx * mx + my * my + kSsimC1, d2 = vx + vy + kSsimC2;
      const float inv = 1.f / (d1 * d2);
      const float s = n1 * n2 * inv;
      ssum += s;
      // derivatives with respect to the shifted statistics (the shift moves the mean term only)
      const float dA = 2.f * my * n2 * inv - 2.f * mx * s / d1 + 2.f * ex * s / d2 - 2.f * ey * n1 * inv;
      const float dB = -s / d2;
      const float dC = 2.f * n1 * inv;
      const size_t o = (size_t)gy * w + gx;
      maps[(0 * 3 + c) * plane + o] = dA;
      maps[(1 * 3 + c) * plane + o] = dB;
      maps[(2 * 3 + c) * plane + o] = dC;
    }
  }
  double d = (double)ssum;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
  if ((t & 63) == 0) red[t >> 6] = d;
  __syncthreads();
  if (t == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void __launch_bounds__(kSsimThreads) ssim_bwd_kernel(const float* __restrict__ img,
                                                                const float* __restrict__ tgt, int w, int h,
                                                                const SsimWeights wt, const float* __restrict__ maps,
                                                                float scale, float* __restrict__ dL) {
  __shared__ float sm[3][kSsimIn][kSsimPitch];
  __shared__ float hs[3][kSsimIn][kSsimT];
  const int t = threadIdx.x;
  const int x0 = blockIdx.x * kSsimT - kSsimR, y0 = blockIdx.y * kSsimT - kSsimR;
  const size_t plane = (size_t)w * h;
  const int ox = t % kSsimT;
#pragma unroll 1
  for (int c = 0; c < 3; ++c) {
    if (c > 0) __syncthreads();
    for (int e = t; e < 3 * kSsimIn * kSsimIn; e += kSsimThreads) {
      const int m = e / (kSsimIn * kSsimIn), rc = e - m * (kSsimIn * kSsimIn);
      const int r = rc / kSsimIn, col = rc - r * kSsimIn;
      const int gx = x0 + col, gy = y0 + r;
      float v = 0.f;                           // the maps are zero outside the image
      if (gx >= 0 && gx < w && gy >= 0 && gy < h) v = maps[(m * 3 + c) * plane + (size_t)gy * w + gx];
      sm[m][r][col] = v;
    }
    __syncthreads();
    for (int i = t; i < kSsimIn * kSsimT; i += kSsimThreads) {
      const int r = i / kSsimT, col = i - r * kSsimT;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
      for (int k = 0; k < kSsimTaps; ++k) {
        const float wk = wt.w[k];
        a0 += wk * sm[0][r][col + k];
        a1 += wk * sm[1][r][col + k];
        a2 += wk * sm[2][r][col + k];
      }
      hs[0][r][col] = a0;
      hs[1][r][col] = a1;
      hs[2][r][col] = a2;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSsimRowsPerThread; ++j) {
      const int oy = t / kSsimT + j * (kSsimThreads / kSsimT);
      float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
      for (int k = 0; k < kSsimTaps; ++k) {
        const float wk = wt.w[k];
        a0 += wk * hs[0][oy + k][ox];
        a1 += wk * hs[1][oy + k][ox];
        a2 += wk * hs[2][oy + k][ox];
      }
      const int gx = x0 + kSsimR + ox, gy = y0 + kSsimR + oy;
      if (gx >= w || gy >= h) continue;
      const size_t o = 3 * ((size_t)gy * w + gx) + c;
      const float xs = img[o] - kSsimShift, ys = tgt[o] - kSsimShift;
      dL[o] = dL[o] - scale * (a0 + 2.f * xs * a1 + ys * a2);
    }
  }
}

// loss += lam (1 - sum / count), the block sums added in a fixed order
__global__ void __launch_bounds__(256) ssim_final_kernel(const double* __restrict__ partial, int nb, double count,
                                                         float lam, float* __restrict__ loss) {
  __shared__ double wsum[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) s += partial[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double total = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    *loss = (float)((double)*loss + (double)lam * (1.0 - total / count));
  }
}

static size_t ssim_blocks(int w, int h) {
  return (size_t)((w + kSsimT - 1) / kSsimT) * (size_t)((h + kSsimT - 1) / kSsimT);
}

size_t ssim_scratch_bytes(int w, int h) {
  const size_t maps = 9 * (size_t)w * h * sizeof(float);
  return ((maps + 255) / 256) * 256 + ssim_blocks(w, h) * sizeof(double);
}

hipError_t launch_ssim_loss(const float* img, const float* target, int w, int h, float lam, void* scratch,
                            float* loss, float* dL, hipStream_t stream) {
  SsimWeights wt;
  double g[kSsimTaps], sum = 0.0;
  for (int k = 0; k < kSsimTaps; ++k) {
    const double d = (double)(k - kSsimR);
    g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[k];
  }
  for (int k = 0; k < kSsimTaps; ++k) wt.w[k] = (float)(g[k] / sum);
  float* maps = reinterpret_cast<float*>(scratch);
  const size_t maps_bytes = ((9 * (size_t)w * h * sizeof(float) + 255) / 256) * 256;
  double* partial = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) + maps_bytes);
  const dim3 grid((w + kSsimT - 1) / kSsimT, (h + kSsimT - 1) / kSsimT);
  const double count = 3.0 * (double)w * (double)h;
  hipLaunchKernelGGL(ssim_fwd_kernel, grid, dim3(kSsimThreads), 0, stream, img, target, w, h, wt, maps, partial);
  hipLaunchKernelGGL(ssim_bwd_kernel, grid, dim3(kSsimThreads), 0, stream, img, target, w, h, wt,
                     (const float*)maps, (float)((double)lam / count), dL);
  hipLaunchKernelGGL(ssim_final_kernel, dim3(1), dim3(256), 0, stream, (const double*)partial,
                     (int)ssim_blocks(w, h), count, lam, loss);
  return hipGetLastError();
}

}  // namespace ges
