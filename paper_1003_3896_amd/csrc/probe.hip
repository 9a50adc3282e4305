// Instrumentation: the issue rate of the pair kernel's FP32 inner loop on this GPU.
//
// k_loop_probe runs the far-tile pair term of the FP32 families (interact32: three differences,
// r^2 in three FMAs, v_rsq_f32, two products, three FMAs; K i-particles per lane) over one LDS tile
// of records, again and again, with the launch bound of the local-mode pair kernel (6 waves per
// SIMD) and nothing else: no staging of tiles, no folds, no near tiles, no work items.  Its SIMD
// cycles per wave-interaction are the floor the full kernel approaches, so 20 cycles (one
// wave-interaction at the FP32 vector peak) divided by them is the ceiling of the pair loop.
#include "../../include/nbody.h"
#include "pair_kernel.h"

namespace nb {
namespace {

constexpr int kProbeTile = 256;

template <int K>
__global__ __launch_bounds__(kBlock, 6) void k_loop_probe(float* out, int reps) {
  __shared__ float4 rec[kProbeTile];
  const int t = threadIdx.x;
  // records on a shell of radius ~1 around the origin, unit weights; i-particles near the origin
  for (int j = t; j < kProbeTile; j += kBlock) {
    const float ph = 0.0245f * (float)j, z = 1.0f - 2.0f * ((float)j + 0.5f) / kProbeTile;
    const float rr = sqrtf(fmaxf(0.0f, 1.0f - z * z));
    rec[j] = make_float4(rr * cosf(ph), rr * sinf(ph), z, 1.0f);
  }
  __syncthreads();
  float xi[K], yi[K], zi[K], xl[K], yl[K], zl[K], ax[K], ay[K], az[K], pt[K];
  int li[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    xi[k] = 1e-3f * (float)(t + 64 * k);
    yi[k] = -xi[k];
    zi[k] = 0.5f * xi[k];
    xl[k] = yl[k] = zl[k] = 0.0f;
    ax[k] = ay[k] = az[k] = pt[k] = 0.0f;
    li[k] = -1;
  }
  const float e2 = 1e-8f;
  for (int r = 0; r < reps; ++r) {
#pragma unroll 2
    for (int u = 0; u < kProbeTile; u += 8) {
#pragma unroll
      for (int v = 0; v < 8; ++v)
        interact32<false, K, false, false, true>(rec[u + v], rec[u + v], xi, yi, zi, xl, yl, zl, e2, ax, ay, az,
                                                 pt, li, 0);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) s += ax[k] + ay[k] + az[k];
  out[(size_t)blockIdx.x * kBlock + t] = s;
}

template <int K>
hipError_t probe_one(float* buf, int blocks, int reps, double* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_loop_probe<K>, dim3(blocks), dim3(kBlock), 0, nullptr, buf, 2);  // warm-up
    e = hipEventRecord(e0, nullptr);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_loop_probe<K>, dim3(blocks), dim3(kBlock), 0, nullptr, buf, reps);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float f = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
  *ms = f;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

}  // namespace
}  // namespace nb

extern "C" int nbody_loop_probe(int device, void* buf, size_t buf_bytes, int k, double* cycles) {
  using namespace nb;
  if (!buf || !cycles || (k != 1 && k != 2) || device < 0) return NB_ERR_ARG;
  int cus = 0, prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
    return NB_ERR_HIP;
  struct Restore {
    int dev;
    ~Restore() {
      if (dev >= 0) (void)hipSetDevice(dev);
    }
  } restore{prev};
  const int blocks = cus * 6;  // 6 waves per SIMD: every block is 4 waves, one per SIMD
  if (buf_bytes < sizeof(float) * (size_t)blocks * kBlock) return NB_ERR_ARG;
  const int reps = 400;
  double ms = 0.0;
  const hipError_t e = k == 1 ? probe_one<1>(static_cast<float*>(buf), blocks, reps, &ms)
                              : probe_one<2>(static_cast<float*>(buf), blocks, reps, &ms);
  if (e != hipSuccess) return NB_ERR_HIP;
  // wave-interactions per SIMD: 6 waves x reps x tile x K; SIMD cycles at the nominal 2.4 GHz
  const double wave_inter = 6.0 * reps * kProbeTile * k;
  *cycles = ms * 1e-3 * 2.4e9 / wave_inter;
  return NB_OK;
}
