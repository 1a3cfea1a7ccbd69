// ssim.hip -- SSIM term of the GES training loss (lambda_ssim L_ssim, Sec. 4.4, Eq. final) and its gradient.
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
// reads the maps (12 B), x, y and the gradient (12 B) and writes the gradient (4 B).  Tiles are dealt to the
// XCDs in bands so the halo re-reads hit L2.
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
constexpr int kSsimStage = (3 * kSsimIn * kSsimIn + kSsimThreads - 1) / kSsimThreads;   // staged values per thread
constexpr int kSsimStage1 = (kSsimIn * kSsimIn + kSsimThreads - 1) / kSsimThreads;     // one channel
constexpr int kSsimGroups = kSsimT / 4;          // 4 neighbouring outputs per thread and pass
constexpr int kSsimSpan = 4 + 2 * kSsimR;         // staged values those 4 outputs read (14)
static_assert(kSsimT * kSsimGroups == kSsimThreads, "one 4-output strip per thread in the pass down");
constexpr float kSsimC1 = 0.01f * 0.01f, kSsimC2 = 0.03f * 0.03f;
constexpr float kSsimShift = 0.5f;

struct SsimWeights {
  float w[kSsimTaps];
};

// Workgroups are dealt to the 8 XCDs in turn (block b runs on XCD b mod 8), and each XCD has its own L2.
// Block b takes tile (b mod 8) * per + b / 8, so every XCD walks one contiguous band of tile rows and the
// halos that neighbouring tiles share are read through the same L2.  Returns -1 for the spare blocks.
__device__ __forceinline__ int ssim_tile(int b, int ntiles) {
  const int per = (ntiles + 7) / 8;
  const int j = b >> 3, tile = (b & 7) * per + j;
  return (j < per && tile < ntiles) ? tile : -1;
}

__global__ void __launch_bounds__(kSsimThreads) ssim_fwd_kernel(const float* __restrict__ img,
                                                                const float* __restrict__ tgt, int w, int h,
                                                                const SsimWeights wt, float* __restrict__ maps,
                                                                double* __restrict__ partial, int tiles_x,
                                                                int ntiles) {
  __shared__ float sx[kSsimIn][kSsimPitch];
  __shared__ float sy[kSsimIn][kSsimPitch];
  __shared__ __align__(16) float hs[5][kSsimIn][kSsimT];
  __shared__ double red[kSsimThreads / 64];
  const int tile = ssim_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int t = threadIdx.x;
  const int x0 = (tile % tiles_x) * kSsimT - kSsimR, y0 = (tile / tiles_x) * kSsimT - kSsimR;
  const size_t plane = (size_t)w * h;
  float ssum = 0.f;
  for (int c = 0; c < 3; ++c) {
    // stage channel c of both images (one channel at a time keeps the block's LDS at 41 KB, three blocks
    // per CU; the other channels' bytes of each line come again from L2); loads first, then the stores
    float ra[kSsimStage1], rb[kSsimStage1];
#pragma unroll
    for (int j = 0; j < kSsimStage1; ++j) {
      const int e = t + j * kSsimThreads;
      ra[j] = 0.f;
      rb[j] = 0.f;
      if (e < kSsimIn * kSsimIn) {
        const int r = e / kSsimIn, col = e - r * kSsimIn;
        const int gx = x0 + col, gy = y0 + r;
        if (gx >= 0 && gx < w && gy >= 0 && gy < h) {
          const size_t o = 3 * ((size_t)gy * w + gx) + c;
          ra[j] = img[o];
          rb[j] = tgt[o];
        }
      }
    }
    __syncthreads();   // the previous channel's horizontal pass has read sx, sy
#pragma unroll
    for (int j = 0; j < kSsimStage1; ++j) {
      const int e = t + j * kSsimThreads;
      if (e < kSsimIn * kSsimIn) {
        const int r = e / kSsimIn, col = e - r * kSsimIn;
        const int gx = x0 + col, gy = y0 + r;
        const bool in = gx >= 0 && gx < w && gy >= 0 && gy < h;   // padding is 0, i.e. -1/2 after the shift
        sx[r][col] = (in ? ra[j] : 0.f) - kSsimShift;
        sy[r][col] = (in ? rb[j] : 0.f) - kSsimShift;
      }
    }
    __syncthreads();
    // across: row r, columns 4g..4g+3 from the 14 staged values they span
    for (int i = t; i < kSsimIn * kSsimGroups; i += kSsimThreads) {
      const int r = i / kSsimGroups, col0 = 4 * (i - r * kSsimGroups);
      float a[kSsimSpan], b[kSsimSpan];
#pragma unroll
      for (int k = 0; k < kSsimSpan; ++k) {
        a[k] = sx[r][col0 + k];
        b[k] = sy[r][col0 + k];
      }
      float m[5][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
        for (int k = 0; k < kSsimTaps; ++k) {
          const float wk = wt.w[k], av = a[q + k], bv = b[q + k];
          m0 = __builtin_fmaf(wk, av, m0);
          m1 = __builtin_fmaf(wk, bv, m1);
          m2 = __builtin_fmaf(wk, av * av, m2);
          m3 = __builtin_fmaf(wk, bv * bv, m3);
          m4 = __builtin_fmaf(wk, av * bv, m4);
        }
        m[0][q] = m0; m[1][q] = m1; m[2][q] = m2; m[3][q] = m3; m[4][q] = m4;
      }
#pragma unroll
      for (int s5 = 0; s5 < 5; ++s5)
        *reinterpret_cast<float4*>(&hs[s5][r][col0]) = make_float4(m[s5][0], m[s5][1], m[s5][2], m[s5][3]);
    }
    __syncthreads();
    // down: column ox, rows 4j..4j+3 from the 14 rows they span
    const int ox = t % kSsimT, oy0 = 4 * (t / kSsimT);
    float st[5][4];
#pragma unroll
    for (int s5 = 0; s5 < 5; ++s5) {
      float col[kSsimSpan];
#pragma unroll
      for (int k = 0; k < kSsimSpan; ++k) col[k] = hs[s5][oy0 + k][ox];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kSsimTaps; ++k) acc = __builtin_fmaf(wt.w[k], col[q + k], acc);
        st[s5][q] = acc;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int oy = oy0 + q;
      const float ex = st[0][q], ey = st[1][q], exx = st[2][q], eyy = st[3][q], exy = st[4][q];
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
  if (t == 0) partial[tile] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void __launch_bounds__(kSsimThreads) ssim_bwd_kernel(const float* __restrict__ img,
                                                                const float* __restrict__ tgt, int w, int h,
                                                                const SsimWeights wt, const float* __restrict__ maps,
                                                                float scale, float* __restrict__ dL, int tiles_x,
                                                                int ntiles) {
  __shared__ float sm[3][kSsimIn][kSsimPitch];
  __shared__ __align__(16) float hs[3][kSsimIn][kSsimT];
  const int tile = ssim_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int t = threadIdx.x;
  const int x0 = (tile % tiles_x) * kSsimT - kSsimR, y0 = (tile / tiles_x) * kSsimT - kSsimR;
  const size_t plane = (size_t)w * h;
  const int ox = t % kSsimT, oy0 = 4 * (t / kSsimT);
  const int gx = x0 + kSsimR + ox;
  // the thread's 4 output pixels (one column, 4 rows): both images read once, all channels
  float xs[4][3], ys[4][3], gacc[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gy = y0 + kSsimR + oy0 + q;
    const bool in = gx < w && gy < h;
    const size_t o = in ? 3 * ((size_t)gy * w + gx) : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xs[q][c] = in ? img[o + c] - kSsimShift : 0.f;
      ys[q][c] = in ? tgt[o + c] - kSsimShift : 0.f;
      gacc[q][c] = 0.f;
    }
  }
#pragma unroll 1
  for (int c = 0; c < 3; ++c) {
    if (c > 0) __syncthreads();
    float rv[kSsimStage];
#pragma unroll
    for (int j = 0; j < kSsimStage; ++j) {     // all loads first, then the LDS stores
      const int e = t + j * kSsimThreads;
      rv[j] = 0.f;                               // the maps are zero outside the image
      if (e < 3 * kSsimIn * kSsimIn) {
        const int m = e / (kSsimIn * kSsimIn), rc = e - m * (kSsimIn * kSsimIn);
        const int r = rc / kSsimIn, col = rc - r * kSsimIn;
        const int gx = x0 + col, gy = y0 + r;
        if (gx >= 0 && gx < w && gy >= 0 && gy < h) rv[j] = maps[(m * 3 + c) * plane + (size_t)gy * w + gx];
      }
    }
#pragma unroll
    for (int j = 0; j < kSsimStage; ++j) {
      const int e = t + j * kSsimThreads;
      if (e < 3 * kSsimIn * kSsimIn) {
        const int m = e / (kSsimIn * kSsimIn), rc = e - m * (kSsimIn * kSsimIn);
        const int r = rc / kSsimIn, col = rc - r * kSsimIn;
        sm[m][r][col] = rv[j];
      }
    }
    __syncthreads();
    for (int i = t; i < kSsimIn * kSsimGroups; i += kSsimThreads) {
      const int r = i / kSsimGroups, col0 = 4 * (i - r * kSsimGroups);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        float v[kSsimSpan];
#pragma unroll
        for (int k = 0; k < kSsimSpan; ++k) v[k] = sm[m][r][col0 + k];
        float o4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float acc = 0.f;
#pragma unroll
          for (int k = 0; k < kSsimTaps; ++k) acc = __builtin_fmaf(wt.w[k], v[q + k], acc);
          o4[q] = acc;
        }
        *reinterpret_cast<float4*>(&hs[m][r][col0]) = make_float4(o4[0], o4[1], o4[2], o4[3]);
      }
    }
    __syncthreads();
    float f[3][4];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      float col[kSsimSpan];
#pragma unroll
      for (int k = 0; k < kSsimSpan; ++k) col[k] = hs[m][oy0 + k][ox];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kSsimTaps; ++k) acc = __builtin_fmaf(wt.w[k], col[q + k], acc);
        f[m][q] = acc;
      }
    }
    // channel c's value of every output (registers picked with constant indices only)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float x_ = c == 0 ? xs[q][0] : (c == 1 ? xs[q][1] : xs[q][2]);
      const float y_ = c == 0 ? ys[q][0] : (c == 1 ? ys[q][1] : ys[q][2]);
      const float g = f[0][q] + 2.f * x_ * f[1][q] + y_ * f[2][q];
      if (c == 0) gacc[q][0] = g;
      else if (c == 1) gacc[q][1] = g;
      else gacc[q][2] = g;
    }
  }
  // one read-modify-write of the three channels of each output pixel
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gy = y0 + kSsimR + oy0 + q;
    if (gx >= w || gy >= h) continue;
    const size_t o = 3 * ((size_t)gy * w + gx);
#pragma unroll
    for (int c = 0; c < 3; ++c) dL[o + c] = dL[o + c] - scale * gacc[q][c];
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
  const int tiles_x = (w + kSsimT - 1) / kSsimT;
  const int ntiles = (int)ssim_blocks(w, h);
  const dim3 grid(8 * ((ntiles + 7) / 8));
  const double count = 3.0 * (double)w * (double)h;
  hipLaunchKernelGGL(ssim_fwd_kernel, grid, dim3(kSsimThreads), 0, stream, img, target, w, h, wt, maps, partial,
                     tiles_x, ntiles);
  hipLaunchKernelGGL(ssim_bwd_kernel, grid, dim3(kSsimThreads), 0, stream, img, target, w, h, wt,
                     (const float*)maps, (float)((double)lam / count), dL, tiles_x, ntiles);
  hipLaunchKernelGGL(ssim_final_kernel, dim3(1), dim3(256), 0, stream, (const double*)partial,
                     (int)ssim_blocks(w, h), count, lam, loss);
  return hipGetLastError();
}

}  // namespace ges
