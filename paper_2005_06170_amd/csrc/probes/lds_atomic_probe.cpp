// Throughput of LDS atomic adds on the current GPU (lanes/clk/CU at 2.4 GHz,
// 256 CUs).  Every index is masked into the LDS array; each workgroup writes
// its own slice of `out`.  Used to set the scatter kernel's roof.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kLds = 8192;

template <typename T, int kMode>
__global__ __launch_bounds__(1024) void probe(T* out, int iters) {
  __shared__ T s[kLds];
  const unsigned tid = threadIdx.x;
  for (unsigned i = tid; i < kLds; i += 1024) s[i] = T(0);
  __syncthreads();
  // kMode 0: distinct banks (stride 37); 1: pseudo-random; 2: 64 lanes on one address
  unsigned base;
  if (kMode == 0) base = (tid * 37u) & (kLds - 1);
  else if (kMode == 1) base = (tid * 2654435761u) >> 19;
  else base = (tid >> 6) * 64u;
  T* p = s + (base & (kLds - 512 - 1));
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 16; ++j) atomicAdd(p + j * 31, T(1));
  }
  __syncthreads();
  out[blockIdx.x * 1024 + tid] = s[tid];
}

template <typename T, int kMode>
void run(const char* name, void* out, int blocks, int iters) {
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  probe<T, kMode><<<blocks, 1024>>>(static_cast<T*>(out), iters);
  (void)hipDeviceSynchronize();
  (void)hipEventRecord(a);
  probe<T, kMode><<<blocks, 1024>>>(static_cast<T*>(out), iters);
  (void)hipEventRecord(b);
  (void)hipEventSynchronize(b);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  const double ops = double(blocks) * 1024 * iters * 16;
  std::printf("| %-30s | %9.3f | %9.1f | %6.2f |\n", name, ms, ops / ms / 1e6, ops / (ms * 1e-3) / 256 / 2.4e9);
}

}  // namespace

int main() {
  const int blocks = 1024, iters = 32;
  void* out = nullptr;
  if (hipMalloc(&out, sizeof(double) * blocks * 1024) != hipSuccess) return 1;
  std::printf("| op | ms | G lane-ops/s | lanes/clk/CU |\n|---|---:|---:|---:|\n");
  run<float, 0>("ds_add_f32, distinct banks", out, blocks, iters / 4);
  run<uint32_t, 0>("ds_add_u32, distinct banks", out, blocks, iters);
  run<uint32_t, 1>("ds_add_u32, random", out, blocks, iters);
  run<uint32_t, 2>("ds_add_u32, one address/wave", out, blocks, iters / 8);
  run<unsigned long long, 0>("ds_add_u64, distinct banks", out, blocks, iters);
  run<double, 0>("ds_add_f64, distinct banks", out, blocks, iters);
  run<double, 1>("ds_add_f64, random", out, blocks, iters);
  const hipError_t e = hipGetLastError();
  std::printf("status: %s\n", hipGetErrorString(e));
  (void)hipFree(out);
  return e == hipSuccess ? 0 : 1;
}
