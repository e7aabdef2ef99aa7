// Device-to-device copy used as the practical bandwidth reference of the roofline
// measurements: a streaming kernel that reads every byte once and writes it once, the access
// pattern of a pull step without its arithmetic. 16-byte non-temporal loads and stores, a
// grid of 8 workgroups per compute unit striding over the buffer.
#include <algorithm>

#include "device_common.h"
#include "lbm.h"

namespace lbm {

typedef float f32x4_t __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kBlock)
k_copy16(const f32x4_t* __restrict__ src, f32x4_t* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void k_copy1(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace lbm

extern "C" int lbm_device_copy(const void* src, void* dst, size_t bytes, void* stream) {
  using namespace lbm;
  if (bytes == 0) return LBM_OK;
  if (!src || !dst) return LBM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) return LBM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 > 0) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t need = (n16 + kBlock - 1) / kBlock;
    const unsigned blocks = (unsigned)std::min<int64_t>(need, (int64_t)cus * 8);
    k_copy16<<<blocks, kBlock, 0, s>>>(static_cast<const f32x4_t*>(src), static_cast<f32x4_t*>(dst), n16);
  }
  const int64_t tail = (int64_t)(bytes % 16);
  if (tail > 0)
    k_copy1<<<1, kBlock, 0, s>>>(static_cast<const unsigned char*>(src) + 16 * n16,
                                 static_cast<unsigned char*>(dst) + 16 * n16, tail);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}
