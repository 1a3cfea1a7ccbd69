// loss.hip -- frequency-modulated L1 loss of GES (Sec. 4.3) and its gradient.
//
// Mask (made per target and omega; the training step remakes it every iteration as omega grows):
//   grey = (r + g + b) / 3, area-down-sampled by 5 (image Laplacian scale 0.2, App. B.2);
//   DoG = G(grey, sigma1) - G(grey, sigma2), sigma2 = 0.1 + 10 omega, sigma1 = 2 sigma2 (Eq. mask),
//   separable normalised Gaussians of radius ceil(3 sigma) with replicated borders;
//   M = |DoG| / max|DoG| > 0.5 (an all-zero mask when max|DoG| <= 1e-5), up-sampled by nearest lookup;
//   for omega <= 0.5, M = 1 - M_(omega+0.5), M_(omega+0.5) taken directly (omega = 0 as the limit from above).
// Loss: L = lam_l1 mean|I - T| + lam_w mean(|I - T| M) (Eq. laplace, Eq. final without the SSIM term),
//   dL/dI = (lam_l1 + lam_w M) sign(I - T) / (3 h w).  The per-block partial sums are added in a
//   fixed order by one block, so the loss is deterministic.
// Memory: the loss reads I, T (12 B/px each) and M (1 B/px) and writes dL/dI (12 B/px): HBM-bound.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "ges_internal.h"

namespace ges {

constexpr int kScale = 5;
constexpr int kMaxTaps = 2 * 64 + 1;   // supports sigma up to 21 (omega <= 1)

// Blur weights of both Gaussians, made on the host and passed by value (they land in the kernel-argument
// segment and are read with scalar loads).
struct MaskWeights {
  float w1[kMaxTaps];
  float w2[kMaxTaps];
  int r1, r2;
};

struct MaskScratch {
  unsigned int maxbits;   // largest |DoG| (non-negative floats order like their bits)
};

size_t freq_mask_scratch_bytes(int w, int h) {
  const size_t wl = (size_t)(w + kScale - 1) / kScale, hl = (size_t)(h + kScale - 1) / kScale;
  return 256 + ((sizeof(MaskScratch) + 255) / 256) * 256 + 4 * wl * hl * sizeof(float) + 256;
}

static void mask_weights(MaskWeights& mw, float s1, float s2) {
  for (int which = 0; which < 2; ++which) {
    const double s = which == 0 ? s1 : s2;
    const int R = (int)std::ceil(3.0 * (double)(which == 0 ? s1 : s2));
    float* w = which == 0 ? mw.w1 : mw.w2;
    double sum = 0.0;
    for (int k = -R; k <= R; ++k) sum += std::exp(-(double)(k * k) / (2.0 * s * s));
    for (int k = -R; k <= R; ++k) w[k + R] = (float)(std::exp(-(double)(k * k) / (2.0 * s * s)) / sum);
    if (which == 0) mw.r1 = R; else mw.r2 = R;
  }
}

__global__ void grey_down_kernel(const float* __restrict__ img, int w, int h, float* __restrict__ low, int wl, int hl,
                                 MaskScratch* __restrict__ ms) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x == 0 && y == 0) ms->maxbits = 0u;   // read only by the later kernels of this mask
  if (x >= wl) return;
  float acc = 0.f;
  int cnt = 0;
  for (int dy = 0; dy < kScale; ++dy) {
    const int yy = y * kScale + dy;
    if (yy >= h) break;
    for (int dx = 0; dx < kScale; ++dx) {
      const int xx = x * kScale + dx;
      if (xx >= w) break;
      const float* p = img + 3 * ((size_t)yy * w + xx);
      acc += (p[0] + p[1] + p[2]) * (1.f / 3.f);
      ++cnt;
    }
  }
  low[(size_t)y * wl + x] = acc / (float)cnt;
}

// horizontal pass of both blurs
__global__ void blur_h_kernel(const MaskWeights mw, const float* __restrict__ low, int wl, int hl,
                              float* __restrict__ h1, float* __restrict__ h2) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= wl) return;
  const float* row = low + (size_t)y * wl;
  float a1 = 0.f, a2 = 0.f;
#pragma unroll 8
  for (int k = -mw.r1; k <= mw.r1; ++k) a1 += mw.w1[k + mw.r1] * row[min(max(x + k, 0), wl - 1)];
#pragma unroll 8
  for (int k = -mw.r2; k <= mw.r2; ++k) a2 += mw.w2[k + mw.r2] * row[min(max(x + k, 0), wl - 1)];
  h1[(size_t)y * wl + x] = a1;
  h2[(size_t)y * wl + x] = a2;
}

// vertical pass, |DoG| and its maximum (a block maximum, then one atomic per block)
__global__ void __launch_bounds__(128) blur_v_dog_kernel(MaskScratch* __restrict__ ms, const MaskWeights mw,
                                                         const float* __restrict__ h1, const float* __restrict__ h2,
                                                         int wl, int hl, float* __restrict__ dog) {
  __shared__ float wmax[2];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  float d = 0.f;
  if (x < wl) {
    float a1 = 0.f, a2 = 0.f;   // unrolled so that several rows' loads are in flight at once
#pragma unroll 8
    for (int k = -mw.r1; k <= mw.r1; ++k) a1 += mw.w1[k + mw.r1] * h1[(size_t)min(max(y + k, 0), hl - 1) * wl + x];
#pragma unroll 8
    for (int k = -mw.r2; k <= mw.r2; ++k) a2 += mw.w2[k + mw.r2] * h2[(size_t)min(max(y + k, 0), hl - 1) * wl + x];
    d = fabsf(a1 - a2);
    dog[(size_t)y * wl + x] = d;
  }
  float m = d;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&ms->maxbits, __float_as_uint(fmaxf(wmax[0], wmax[1])));
}

__global__ void mask_up_kernel(const MaskScratch* __restrict__ ms, const float* __restrict__ dog, int wl, int w, int h,
                               int invert, uint8_t* __restrict__ mask) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= w) return;
  const float m = __uint_as_float(ms->maxbits);
  uint8_t bit = 0;
  if (m > 1e-5f) bit = (dog[(size_t)(y / kScale) * wl + x / kScale] / m) > 0.5f ? 1 : 0;
  mask[(size_t)y * w + x] = invert ? (uint8_t)(1 - bit) : bit;
}

hipError_t launch_freq_mask(const float* target, int w, int h, float omega, void* scratch, uint8_t* mask,
                            hipStream_t stream) {
  const bool invert = omega <= 0.5f;
  const float om = invert ? omega + 0.5f : omega;
  const float s2 = 0.1f + 10.f * om, s1 = 2.f * s2;
  const int wl = (w + kScale - 1) / kScale, hl = (h + kScale - 1) / kScale;
  char* base = reinterpret_cast<char*>(scratch);
  MaskScratch* ms = reinterpret_cast<MaskScratch*>(base);
  float* low = reinterpret_cast<float*>(base + ((sizeof(MaskScratch) + 255) / 256) * 256);
  float* h1 = low + (size_t)wl * hl;
  float* h2 = h1 + (size_t)wl * hl;
  float* dog = h2 + (size_t)wl * hl;
  MaskWeights mw;
  mask_weights(mw, s1, s2);
  const dim3 gl((wl + 127) / 128, hl);
  hipLaunchKernelGGL(grey_down_kernel, gl, dim3(128), 0, stream, target, w, h, low, wl, hl, ms);
  hipLaunchKernelGGL(blur_h_kernel, gl, dim3(128), 0, stream, mw, low, wl, hl, h1, h2);
  hipLaunchKernelGGL(blur_v_dog_kernel, gl, dim3(128), 0, stream, ms, mw, h1, h2, wl, hl, dog);
  hipLaunchKernelGGL(mask_up_kernel, dim3((w + 255) / 256, h), dim3(256), 0, stream, ms, dog, wl, w, h,
                     invert ? 1 : 0, mask);
  return hipGetLastError();
}

// ---- the mask with library-held scratch (no scratch argument, no allocation) -------------------
// One fixed array per device; its device address is looked up once per device, with that device
// current, and kept.  Host code never passes the array's own name to a kernel (on the host that name is a
// stand-in, not a device address): every use goes through the looked-up pointer.
constexpr size_t kMaskStaticBytes = GES_MASK_STATIC_SCRATCH_BYTES;
constexpr int kMaxStaticDevices = 64;
static __device__ __align__(256) unsigned char mask_static_scratch[kMaskStaticBytes];

namespace {
std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices] = {};
}  // namespace

size_t freq_mask_static_capacity() { return kMaskStaticBytes; }

hipError_t launch_freq_mask_static(const float* target, int w, int h, float omega, uint8_t* mask,
                                   hipStream_t stream) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxStaticDevices) return hipErrorInvalidDevice;
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
      e = hipGetSymbolAddress(&g_static_ptr[dev], HIP_SYMBOL(mask_static_scratch));
      if (e != hipSuccess) {
        g_static_ptr[dev] = nullptr;
        return e;
      }
    }
    ptr = g_static_ptr[dev];
  }
  // the maximum word the scratch holds is cleared by the first kernel of the mask, so nothing else
  // has to start at zero
  return launch_freq_mask(target, w, h, omega, ptr, mask, stream);
}

constexpr int kLossThreads = 256;
constexpr int kLossBlocks = 1024;

__global__ void __launch_bounds__(kLossThreads) loss_kernel(const float* __restrict__ img,
                                                            const float* __restrict__ tgt,
                                                            const uint8_t* __restrict__ mask, int64_t npix,
                                                            float lam_l1, float lam_w, float* __restrict__ dL,
                                                            float* __restrict__ partial) {
  __shared__ float red[kLossThreads / 64];
  const float inv_n = 1.f / (3.f * (float)npix);
  float acc = 0.f;
  for (int64_t p = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; p < npix; p += (int64_t)gridDim.x * kLossThreads) {
    const float wgt = lam_l1 + (mask ? lam_w * (float)mask[p] : 0.f);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float d = img[3 * p + c] - tgt[3 * p + c];
      acc = __builtin_fmaf(wgt, fabsf(d), acc);
      const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
      dL[3 * p + c] = wgt * sg * inv_n;
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int k = 0; k < kLossThreads / 64; ++k) s += red[k];
    partial[blockIdx.x] = s;
  }
}

// Sum of the block partials in binary64, in a fixed order: 256 strided partial sums, then a fixed
// butterfly within each wave and the four wave sums in order.
__global__ void __launch_bounds__(256) loss_final_kernel(const float* __restrict__ partial, int nb, float scale,
                                                         float* __restrict__ out) {
  __shared__ double wsum[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) s += (double)partial[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (float)((((wsum[0] + wsum[1]) + wsum[2]) + wsum[3]) * (double)scale);
}

size_t loss_scratch_bytes() { return kLossBlocks * sizeof(float); }

hipError_t launch_loss(const float* img, const float* target, const uint8_t* mask, int w, int h, float lam_l1,
                       float lam_w, void* scratch, float* loss_out, float* dL_dimg, hipStream_t stream) {
  const int64_t npix = (int64_t)w * h;
  float* partial = reinterpret_cast<float*>(scratch);
  const int nb = (int)std::min<int64_t>(kLossBlocks, (npix + kLossThreads - 1) / kLossThreads);
  hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(kLossThreads), 0, stream, img, target, mask, npix, lam_l1, lam_w,
                     dL_dimg, partial);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, stream, partial, nb, 1.f / (3.f * (float)npix), loss_out);
  return hipGetLastError();
}

__global__ void zero_kernel(uint4* p, size_t n16, uint8_t* tail, size_t ntail) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16;
  const unsigned blocks = (unsigned)std::min<size_t>(4096, (n16 + 255) / 256 + 1);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, stream, reinterpret_cast<uint4*>(p), n16,
                     reinterpret_cast<uint8_t*>(p) + n16 * 16, bytes - n16 * 16);
  return hipGetLastError();
}

}  // namespace ges
