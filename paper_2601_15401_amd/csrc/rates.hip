// Instruction-rate and bandwidth probe for the roofline denominators of the
// k-input multiply on gfx950.
//
// The ring arithmetic of the multiply is 32-bit integer work: Shoup and
// Montgomery products (v_mul_lo_u32, v_mul_hi_u32), 64-bit multiply-adds of
// the basis conversion and key products (v_mad_u64_u32), and the additions
// and selections around them.  The only matrix-core form that could carry an
// exact basis conversion is the int8 product with int32 accumulation.  This
// program measures, on the current device, the issue rate of each of those
// instructions (independent chains in every lane, enough waves to fill every
// SIMD) and the bandwidth of a plain device copy, and prints one JSON line.
//
// Lane-ops per CU per clock are reported at the device's reported peak clock
// and at the nominal 2.4 GHz.  Nothing here is part of the multiply.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <string>
#include <vector>

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;  // independent dependency chains per lane

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
      return 1;                                                               \
    }                                                                         \
  } while (0)

enum Op { OP_ADD, OP_MUL_LO, OP_MUL_HI, OP_MAD64, OP_COUNT_VALU };

template <int OP>
__global__ __launch_bounds__(kThreads) void k_valu(uint32_t* out, int iters, uint32_t c) {
  uint32_t x[kChains];
  uint64_t w[kChains];
#pragma unroll
  for (int i = 0; i < kChains; i++) {
    x[i] = threadIdx.x * 7919u + i * 104729u + blockIdx.x;
    w[i] = x[i];
  }
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int i = 0; i < kChains; i++) {
      if constexpr (OP == OP_ADD) {
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[i]) : "v"(c));
      } else if constexpr (OP == OP_MUL_LO) {
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[i]) : "v"(c));
      } else if constexpr (OP == OP_MUL_HI) {
        asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[i]) : "v"(c));
      } else {
        uint64_t cy;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(w[i]), "=s"(cy) : "v"(x[i]), "v"(c));
      }
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kChains; i++) s += x[i] + (uint32_t)w[i] + (uint32_t)(w[i] >> 32);
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// SHAPE 0: v_mfma_i32_16x16x64_i8 (16 x 16 x 64 MACs per wave instruction);
// SHAPE 1: v_mfma_i32_32x32x32_i8 (32 x 32 x 32).  Four independent
// accumulators per wave keep the matrix pipeline busy.
template <int SHAPE>
__global__ __launch_bounds__(kThreads) void k_mfma(int* out, int iters, int seed) {
  v4i a = {seed + (int)threadIdx.x, seed ^ 0x01020304, seed * 3, 0x7f7f7f7f};
  v4i b = {(int)threadIdx.x * 5, seed, 0x11223344, (int)blockIdx.x};
  if constexpr (SHAPE == 0) {
    v4i acc[4] = {};
    for (int it = 0; it < iters; it++) {
#pragma unroll
      for (int i = 0; i < 4; i++) acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[i], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) s += acc[i].x + acc[i].y + acc[i].z + acc[i].w;
    out[blockIdx.x * kThreads + threadIdx.x] = s;
  } else {
    v16i acc[4] = {};
    for (int it = 0; it < iters; it++) {
#pragma unroll
      for (int i = 0; i < 4; i++) acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[i], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = 0; j < 16; j++) s += acc[i][j];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
  }
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                   size_t n) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

struct Timer {
  hipEvent_t a, b;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

}  // namespace

int main(int argc, char** argv) {
  int dev = 0;
  CHECK(hipSetDevice(dev));
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, dev));
  const int cus = prop.multiProcessorCount;
  const double clk_ghz = prop.clockRate / 1e6;  // kHz -> GHz
  const int blocks = cus * 8;                     // eight 256-thread workgroups per CU: 8 waves per SIMD
  uint32_t* out = nullptr;
  CHECK(hipMalloc(&out, (size_t)blocks * kThreads * 4));
  Timer t;
  std::string json = "{";
  char buf[512];
  snprintf(buf, sizeof buf, "\"device\": \"%s\", \"arch\": \"%s\", \"cus\": %d, \"peak_clock_ghz\": %.3f", prop.name,
           prop.gcnArchName, cus, clk_ghz);
  json += buf;

  const char* names[OP_COUNT_VALU] = {"v_add_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32"};
  const int iters = 4096;
  for (int op = 0; op < OP_COUNT_VALU; op++) {
    auto launch = [&]() {
      switch (op) {
        case OP_ADD: k_valu<OP_ADD><<<blocks, kThreads>>>(out, iters, 3u); break;
        case OP_MUL_LO: k_valu<OP_MUL_LO><<<blocks, kThreads>>>(out, iters, 0x9E3779B9u); break;
        case OP_MUL_HI: k_valu<OP_MUL_HI><<<blocks, kThreads>>>(out, iters, 0x9E3779B9u); break;
        default: k_valu<OP_MAD64><<<blocks, kThreads>>>(out, iters, 0x9E3779B9u); break;
      }
    };
    launch();
    CHECK(hipDeviceSynchronize());
    float best = 1e30f;
    for (int rep = 0; rep < 5; rep++) {
      CHECK(hipEventRecord(t.a));
      launch();
      CHECK(hipEventRecord(t.b));
      CHECK(hipEventSynchronize(t.b));
      float ms;
      CHECK(hipEventElapsedTime(&ms, t.a, t.b));
      best = ms < best ? ms : best;
    }
    const double lane_ops = (double)blocks * kThreads * iters * kChains;
    const double rate = lane_ops / (best * 1e-3);
    snprintf(buf, sizeof buf,
             ", \"%s\": {\"lane_ops_per_s\": %.4e, \"per_cu_clk_at_peak_clock\": %.2f, \"per_cu_clk_at_2.4GHz\": %.2f}",
             names[op], rate, rate / (cus * clk_ghz * 1e9), rate / (cus * 2.4e9));
    json += buf;
  }

  const char* mnames[2] = {"v_mfma_i32_16x16x64_i8", "v_mfma_i32_32x32x32_i8"};
  const double macs_per_inst[2] = {16.0 * 16 * 64, 32.0 * 32 * 32};
  const int miters = 2048;
  for (int sh = 0; sh < 2; sh++) {
    auto launch = [&]() {
      if (sh == 0)
        k_mfma<0><<<blocks, kThreads>>>(reinterpret_cast<int*>(out), miters, 12345);
      else
        k_mfma<1><<<blocks, kThreads>>>(reinterpret_cast<int*>(out), miters, 12345);
    };
    launch();
    CHECK(hipDeviceSynchronize());
    float best = 1e30f;
    for (int rep = 0; rep < 5; rep++) {
      CHECK(hipEventRecord(t.a));
      launch();
      CHECK(hipEventRecord(t.b));
      CHECK(hipEventSynchronize(t.b));
      float ms;
      CHECK(hipEventElapsedTime(&ms, t.a, t.b));
      best = ms < best ? ms : best;
    }
    const double waves = (double)blocks * (kThreads / 64);
    const double ops = waves * miters * 4 * macs_per_inst[sh] * 2;  // one MAC = two ops
    const double rate = ops / (best * 1e-3);
    snprintf(buf, sizeof buf,
             ", \"%s\": {\"int8_ops_per_s\": %.4e, \"macs_per_cu_clk_at_peak_clock\": %.1f, "
             "\"macs_per_cu_clk_at_2.4GHz\": %.1f}",
             mnames[sh], rate, rate / 2 / (cus * clk_ghz * 1e9), rate / 2 / (cus * 2.4e9));
    json += buf;
  }

  const size_t bytes = (size_t)1 << 30;
  void *src = nullptr, *dst = nullptr;
  CHECK(hipMalloc(&src, bytes));
  CHECK(hipMalloc(&dst, bytes));
  CHECK(hipMemset(src, 1, bytes));
  const size_t n4 = bytes / 16;
  const int cblocks = cus * 16;
  k_copy<<<cblocks, kThreads>>>((const u32x4*)src, (u32x4*)dst, n4);
  CHECK(hipDeviceSynchronize());
  float best = 1e30f;
  for (int rep = 0; rep < 5; rep++) {
    CHECK(hipEventRecord(t.a));
    k_copy<<<cblocks, kThreads>>>((const u32x4*)src, (u32x4*)dst, n4);
    CHECK(hipEventRecord(t.b));
    CHECK(hipEventSynchronize(t.b));
    float ms;
    CHECK(hipEventElapsedTime(&ms, t.a, t.b));
    best = ms < best ? ms : best;
  }
  snprintf(buf, sizeof buf, ", \"copy_1GiB\": {\"bytes_moved\": %zu, \"us\": %.1f, \"GB_per_s\": %.1f}", 2 * bytes,
           best * 1e3, 2.0 * bytes / (best * 1e-3) / 1e9);
  json += buf;
  json += "}";
  printf("%s\n", json.c_str());
  CHECK(hipFree(src));
  CHECK(hipFree(dst));
  CHECK(hipFree(out));
  (void)argc;
  (void)argv;
  return 0;
}
