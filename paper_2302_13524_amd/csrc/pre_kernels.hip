// Preprocessing of the camera image stack (Sec. 2.2, the paragraph after
// Algorithm 1). The kept pixels of an H x W image are its 1-based odd rows and
// columns (0-based even), a (H/2) x (W/2) grid indexed q = y (W/2) + x.
//  * energy: per kept pixel, the intensity summed over all images (FP64),
//    in image chunks (partials) and a fixed-order final sum;
//  * mask: the smallest brightest-first set of kept pixels whose summed
//    intensity first reaches frac of the total (ties by raster index), as
//    ascending raster indices: one workgroup sorts the (energy, index) pairs
//    in LDS (bitonic), scans the sorted energies and compacts the flags;
//  * gather: the per-pixel rows out[p][i] (i = image = measurement index),
//    a transpose through LDS tiles of 64 images x 256 pixels so that both the
//    image reads and the row writes are contiguous.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pre.hpp"

namespace tmk {

namespace {

__device__ __forceinline__ float pix_val(const void* s, int u16, size_t idx) {
  return u16 ? (float)((const uint16_t*)s)[idx] : ((const float*)s)[idx];
}

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Scalar form: grid (ceil(npix / 256), nchunks), thread = kept pixel, loop
// over the chunk's images.
__global__ void __launch_bounds__(256) k_energy_part(const void* stack, int u16, int64_t n_img, int H, int W,
                                                     int64_t chunk, double* partial) {
  const int npix = (H / 2) * (W / 2);
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= npix) return;
  const int y = q / (W / 2), x = q - y * (W / 2);
  const size_t off = (size_t)(2 * y) * W + 2 * x;
  const int64_t i0 = (int64_t)blockIdx.y * chunk;
  const int64_t i1 = (i0 + chunk < n_img) ? i0 + chunk : n_img;
  double s = 0.0;
  for (int64_t i = i0; i < i1; ++i) s += (double)pix_val(stack, u16, (size_t)i * H * W + off);
  partial[(size_t)blockIdx.y * npix + q] = s;
}

// Vector form (16-byte rows segments): a thread owns one 16-byte segment of an
// even row, i.e. KP kept pixels (4 for uint16, 2 for float), and loops over
// the chunk's images with one 16-byte load each. grid (ceil(nseg / 256),
// nchunks), nseg = (H/2) * (W * sizeof / 16).
template <bool U16>
__global__ void __launch_bounds__(256) k_energy_vec(const void* stack, int64_t n_img, int H, int W, int64_t chunk,
                                                    double* partial) {
  constexpr int EPS = U16 ? 8 : 4;  // elements per segment
  constexpr int KP = EPS / 2;       // kept pixels per segment
  const int segs = W / EPS, npix = (H / 2) * (W / 2);
  const int sgi = blockIdx.x * 256 + threadIdx.x;
  if (sgi >= (H / 2) * segs) return;
  const int y = sgi / segs, sx = sgi - y * segs;
  const size_t off = (size_t)(2 * y) * W + (size_t)sx * EPS;
  const size_t plane = (size_t)H * W;
  const int64_t i0 = (int64_t)blockIdx.y * chunk;
  const int64_t i1 = (i0 + chunk < n_img) ? i0 + chunk : n_img;
  double acc[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) acc[k] = 0.0;
#pragma unroll 4
  for (int64_t i = i0; i < i1; ++i) {
    const uint4 v = *(const uint4*)((const char*)stack + (i * plane + off) * (U16 ? 2 : 4));
    if (U16) {
      acc[0] += (double)(v.x & 0xffffu);
      acc[1] += (double)(v.y & 0xffffu);
      acc[2] += (double)(v.z & 0xffffu);
      acc[3] += (double)(v.w & 0xffffu);
    } else {
      acc[0] += (double)__uint_as_float(v.x);
      acc[1] += (double)__uint_as_float(v.z);
    }
  }
  const int q = y * (W / 2) + sx * KP;
#pragma unroll
  for (int k = 0; k < KP; ++k) partial[(size_t)blockIdx.y * npix + q + k] = acc[k];
}

__global__ void __launch_bounds__(256) k_energy_final(const double* partial, int nchunks, int npix, double* energy) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= npix) return;
  double s = 0.0;
#pragma unroll 8
  for (int c = 0; c < nchunks; ++c) s += partial[(size_t)c * npix + q];
  energy[q] = s;
}

constexpr int MWG = 1024;

// a before b in the brightest-first order (ties: smaller raster index first)
__device__ __forceinline__ bool before(double ea, int ia, double eb, int ib) {
  return ea > eb || (ea == eb && ia < ib);
}

__global__ void __launch_bounds__(MWG) k_mask(const double* energy, int npix, double frac, int32_t* pix,
                                             int32_t* count_dev) {
  __shared__ double key[PRE_MASK_MAX];  // energies; after the sort, their running sums; then flags
  __shared__ int idx[PRE_MASK_MAX];
  __shared__ double red[MWG / 64];
  __shared__ int first;
  int M = 1;
  while (M < npix) M <<= 1;
  for (int t = threadIdx.x; t < M; t += MWG) {
    key[t] = (t < npix) ? energy[t] : -INFINITY;
    idx[t] = t;
  }
  if (threadIdx.x == 0) first = M;
  __syncthreads();
  // bitonic sort into the brightest-first order
  for (int k = 2; k <= M; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < M; t += MWG) {
        const int u = t ^ j;
        if (u > t) {
          const bool up = (t & k) == 0;
          const bool sw = up ? before(key[u], idx[u], key[t], idx[t]) : before(key[t], idx[t], key[u], idx[u]);
          if (sw) {
            double e = key[t];
            key[t] = key[u];
            key[u] = e;
            int i = idx[t];
            idx[t] = idx[u];
            idx[u] = i;
          }
        }
      }
      __syncthreads();
    }
  }
  // total (sum of the sorted energies) and the inclusive running sums, in place
  for (int t = threadIdx.x; t < M; t += MWG)
    if (t >= npix) key[t] = 0.0;
  __syncthreads();
  double tot = 0.0;
  for (int t = threadIdx.x; t < npix; t += MWG) tot += key[t];
  for (int off = 32; off >= 1; off >>= 1) tot += __shfl_xor(tot, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tot;
  __syncthreads();
  double total = 0.0;
  for (int w = 0; w < MWG / 64; ++w) total += red[w];
  for (int d = 1; d < M; d <<= 1) {  // Hillis-Steele scan, two phases per step
    double v[PRE_MASK_MAX / MWG];
    for (int c = 0, t = threadIdx.x; t < M; t += MWG, ++c) v[c] = (t >= d) ? key[t - d] : 0.0;
    __syncthreads();
    for (int c = 0, t = threadIdx.x; t < M; t += MWG, ++c) key[t] += v[c];
    __syncthreads();
  }
  // count = (first position whose running sum reaches frac * total) + 1
  const double thr = frac * total;
  for (int t = threadIdx.x; t < npix; t += MWG)
    if (key[t] >= thr) atomicMin(&first, t);
  __syncthreads();
  const int count = (total > 0.0) ? ((first < npix) ? first + 1 : npix) : 0;
  // flags by raster index (over the no longer needed running sums), then compaction
  int* flag = (int*)key;
  for (int t = threadIdx.x; t < M; t += MWG) flag[t] = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < count; t += MWG) flag[idx[t]] = 1;
  __syncthreads();
  for (int d = 1; d < M; d <<= 1) {  // inclusive scan of the flags
    int v[PRE_MASK_MAX / MWG];
    for (int c = 0, t = threadIdx.x; t < M; t += MWG, ++c) v[c] = (t >= d) ? flag[t - d] : 0;
    __syncthreads();
    for (int c = 0, t = threadIdx.x; t < M; t += MWG, ++c) flag[t] += v[c];
    __syncthreads();
  }
  for (int t = threadIdx.x; t < npix; t += MWG) {
    const int before_t = (t > 0) ? flag[t - 1] : 0;
    if (flag[t] != before_t) pix[before_t] = t;
  }
  if (threadIdx.x == 0) *count_dev = count;
}

constexpr int GT_I = 32, GT_P = 256;

// grid (ceil(P / 256), ceil(n_img / 32)), 256 threads; the LDS tile (32 images
// x 256 pixels, 33 KiB) leaves room for four workgroups per CU
__global__ void __launch_bounds__(256) k_gather(const void* stack, int u16, int64_t n_img, int H, int W,
                                               const int32_t* pix, int P, void* out, int out_bf16) {
  __shared__ float tile[GT_I][GT_P + 1];
  const int p0 = blockIdx.x * GT_P;
  const int64_t i0 = (int64_t)blockIdx.y * GT_I;
  const int p = p0 + threadIdx.x;
  size_t off = 0;
  if (p < P) {
    const int q = pix[p];
    const int y = q / (W / 2), x = q - y * (W / 2);
    off = (size_t)(2 * y) * W + 2 * x;
  }
  const size_t plane = (size_t)H * W;
#pragma unroll 8
  for (int r = 0; r < GT_I; ++r) {
    const int64_t i = i0 + r;
    tile[r][threadIdx.x] = (p < P && i < n_img) ? pix_val(stack, u16, (size_t)i * plane + off) : 0.f;
  }
  __syncthreads();
  // 4 consecutive images per thread, 8 threads per pixel, 32 pixels per pass
  const int r4 = (threadIdx.x & 7) * 4;
  for (int pp = threadIdx.x >> 3; pp < GT_P; pp += 32) {
    const int pg = p0 + pp;
    if (pg >= P) break;
    const int64_t i = i0 + r4;
    const size_t o = (size_t)pg * n_img + i;
    const float v0 = tile[r4][pp], v1 = tile[r4 + 1][pp], v2 = tile[r4 + 2][pp], v3 = tile[r4 + 3][pp];
    if (i + 3 < n_img && (o & 3) == 0 && ((uintptr_t)out % 16) == 0) {
      if (out_bf16) {
        uint2 w;
        w.x = (uint32_t)to_bf16(v0) | ((uint32_t)to_bf16(v1) << 16);
        w.y = (uint32_t)to_bf16(v2) | ((uint32_t)to_bf16(v3) << 16);
        *(uint2*)((uint16_t*)out + o) = w;
      } else {
        *(float4*)((float*)out + o) = make_float4(v0, v1, v2, v3);
      }
    } else {
      const float v[4] = {v0, v1, v2, v3};
      for (int k = 0; k < 4; ++k) {
        if (i + k < n_img) {
          if (out_bf16) ((uint16_t*)out)[o + k] = to_bf16(v[k]);
          else ((float*)out)[o + k] = v[k];
        }
      }
    }
  }
}

}  // namespace

// The vector form needs whole 16-byte segments per row and a 16-byte aligned stack.
static bool energy_vec(const void* stack, int u16, int W) {
  return (W % (u16 ? 8 : 4)) == 0 && ((uintptr_t)stack % 16) == 0;
}

static int energy_threads(const void* stack, int u16, int H, int W) {
  return energy_vec(stack, u16, W) ? (H / 2) * (W / (u16 ? 8 : 4)) : (H / 2) * (W / 2);
}

int pre_energy_chunks(const void* stack, int u16, int64_t n_img, int H, int W) {
  // about 1024 workgroups, at least 32 images per chunk, at most 128 chunks (the
  // final pass adds the chunks of each pixel in order)
  const int blocks_x = (energy_threads(stack, u16, H, W) + 255) / 256;
  int64_t c = (1024 + blocks_x - 1) / blocks_x;
  const int64_t maxc = (n_img + 31) / 32;
  if (c > maxc) c = maxc;
  if (c > 128) c = 128;
  return (int)(c < 1 ? 1 : c);
}

int launch_pre_energy(const void* stack, int u16, int64_t n_img, int H, int W, double* partial, int nchunks,
                      double* energy, void* stream) {
  const int npix = (H / 2) * (W / 2);
  const int64_t chunk = (n_img + nchunks - 1) / nchunks;
  hipStream_t s = (hipStream_t)stream;
  dim3 g((energy_threads(stack, u16, H, W) + 255) / 256, nchunks);
  if (!energy_vec(stack, u16, W)) k_energy_part<<<g, 256, 0, s>>>(stack, u16, n_img, H, W, chunk, partial);
  else if (u16) k_energy_vec<true><<<g, 256, 0, s>>>(stack, n_img, H, W, chunk, partial);
  else k_energy_vec<false><<<g, 256, 0, s>>>(stack, n_img, H, W, chunk, partial);
  k_energy_final<<<(npix + 255) / 256, 256, 0, s>>>(partial, nchunks, npix, energy);
  return (int)hipGetLastError();
}

int launch_pre_mask(const double* energy, int npix, double frac, int32_t* pix, int32_t* count_dev, void* stream) {
  k_mask<<<1, MWG, 0, (hipStream_t)stream>>>(energy, npix, frac, pix, count_dev);
  return (int)hipGetLastError();
}

int launch_pre_gather(const void* stack, int u16, int64_t n_img, int H, int W, const int32_t* pix, int P, void* out,
                      int out_bf16, void* stream) {
  if (P <= 0 || n_img <= 0) return 0;
  dim3 g((P + GT_P - 1) / GT_P, (unsigned)((n_img + GT_I - 1) / GT_I));
  k_gather<<<g, 256, 0, (hipStream_t)stream>>>(stack, u16, n_img, H, W, pix, P, out, out_bf16);
  return (int)hipGetLastError();
}

}  // namespace tmk
