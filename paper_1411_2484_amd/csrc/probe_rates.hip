// Instruction-rate probe for gfx950: issue rate of the VALU instruction
// classes the generator uses (32-bit integer multiplies, v_mad_u64_u32,
// carries, selects, FP64 FMA / reciprocal / IEEE divide) and the streaming
// store bandwidth.  Each rate kernel runs 8 independent chains per lane of
// one instruction for 2048 x 4 iterations on 8 waves per SIMD; the rate is
// reported as lane-operations per compute unit per clock (64 = one wave64
// instruction per clock per CU).  The numbers price the roofline model of
// the generation kernels.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <vector>

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { \
  fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); exit(1);} } while (0)

constexpr int ITER = 2048;

#define BODY8(STMT) STMT(0) STMT(1) STMT(2) STMT(3) STMT(4) STMT(5) STMT(6) STMT(7)

// each kernel: 8 independent chains, ITER iterations, result folded into out
#define KERN_U32(NAME, ASM)                                                          \
__global__ void __launch_bounds__(256) NAME(uint32_t *out, uint32_t seed) {          \
  uint32_t b = seed ^ threadIdx.x;                                                   \
  uint32_t x0 = b+1, x1 = b+2, x2 = b+3, x3 = b+4, x4 = b+5, x5 = b+6, x6 = b+7, x7 = b+8; \
  for (int it = 0; it < ITER; ++it) {                                                \
    _Pragma("unroll")                                                                \
    for (int u = 0; u < 4; ++u) {                                                    \
      asm volatile(ASM : "+v"(x0) : "v"(b)); asm volatile(ASM : "+v"(x1) : "v"(b));  \
      asm volatile(ASM : "+v"(x2) : "v"(b)); asm volatile(ASM : "+v"(x3) : "v"(b));  \
      asm volatile(ASM : "+v"(x4) : "v"(b)); asm volatile(ASM : "+v"(x5) : "v"(b));  \
      asm volatile(ASM : "+v"(x6) : "v"(b)); asm volatile(ASM : "+v"(x7) : "v"(b));  \
    }                                                                                \
  }                                                                                  \
  out[blockIdx.x * blockDim.x + threadIdx.x] = x0^x1^x2^x3^x4^x5^x6^x7;              \
}

KERN_U32(k_add_u32,     "v_add_u32 %0, %0, %1")
KERN_U32(k_mul_lo_u32,  "v_mul_lo_u32 %0, %0, %1")
KERN_U32(k_mul_hi_u32,  "v_mul_hi_u32 %0, %0, %1")
KERN_U32(k_mul_u32_u24, "v_mul_u32_u24 %0, %0, %1")
KERN_U32(k_mul_hi_u32_u24, "v_mul_hi_u32_u24 %0, %0, %1")
KERN_U32(k_alignbit,    "v_alignbit_b32 %0, %0, %1, 31")
KERN_U32(k_min_u32,     "v_min_u32 %0, %0, %1")
KERN_U32(k_and_b32,     "v_and_b32 %0, %0, %1")
KERN_U32(k_cvt_f32_u32, "v_cvt_f32_u32 %0, %0")
KERN_U32(k_mad_u32_u24, "v_mad_u32_u24 %0, %0, %1, %1")
KERN_U32(k_add3_u32,    "v_add3_u32 %0, %0, %1, %1")

// carry chain: v_add_co_u32 + v_addc_co_u32 pairs (counts 2 instructions per statement)
__global__ void __launch_bounds__(256) k_addc(uint32_t *out, uint32_t seed) {
  uint32_t b = seed ^ threadIdx.x;
  uint32_t lo[8], hi[8];
  for (int i = 0; i < 8; ++i) { lo[i] = b + i; hi[i] = b * 3 + i; }
  for (int it = 0; it < ITER; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        asm volatile("v_add_co_u32 %0, vcc, %0, %2\n\tv_addc_co_u32 %1, vcc, %1, %2, vcc"
                     : "+v"(lo[i]), "+v"(hi[i]) : "v"(b) : "vcc");
    }
  }
  uint32_t r = 0;
  for (int i = 0; i < 8; ++i) r ^= lo[i] ^ hi[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// v_cndmask with vcc produced once outside the loop
__global__ void __launch_bounds__(256) k_cndmask(uint32_t *out, uint32_t seed) {
  uint32_t b = seed ^ threadIdx.x;
  uint32_t x[8];
  for (int i = 0; i < 8; ++i) x[i] = b + i;
  for (int it = 0; it < ITER; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        asm volatile("v_cmp_gt_u32 vcc, %0, %1\n\tv_cndmask_b32 %0, %0, %1, vcc" : "+v"(x[i]) : "v"(b) : "vcc");
    }
  }
  uint32_t r = 0;
  for (int i = 0; i < 8; ++i) r ^= x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// v_mad_u64_u32: 64-bit accumulators
__global__ void __launch_bounds__(256) k_mad_u64_u32(uint32_t *out, uint32_t seed) {
  uint32_t b = seed ^ threadIdx.x;
  uint64_t x[8];
  for (int i = 0; i < 8; ++i) x[i] = (uint64_t)b * (i + 1);
  for (int it = 0; it < ITER; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %1, %0" : "+v"(x[i]) : "v"(b) : "vcc");
    }
  }
  uint64_t r = 0;
  for (int i = 0; i < 8; ++i) r ^= x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(r ^ (r >> 32));
}

// interleave: one mul_hi + 3 adds (checks whether cheap ops overlap the multiplier)
__global__ void __launch_bounds__(256) k_mulhi_plus3add(uint32_t *out, uint32_t seed) {
  uint32_t b = seed ^ threadIdx.x;
  uint32_t x[8], y[8];
  for (int i = 0; i < 8; ++i) { x[i] = b + i; y[i] = b ^ i; }
  for (int it = 0; it < ITER; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        asm volatile("v_mul_hi_u32 %0, %0, %2\n\tv_add_u32 %1, %1, %2\n\tv_add_u32 %1, %1, %2\n\tv_add_u32 %1, %1, %2"
                     : "+v"(x[i]), "+v"(y[i]) : "v"(b));
    }
  }
  uint32_t r = 0;
  for (int i = 0; i < 8; ++i) r ^= x[i] ^ y[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

#define KERN_F64(NAME, ASM)                                                         \
__global__ void __launch_bounds__(256) NAME(uint32_t *out, uint32_t seed) {          \
  double b = 1.0 + 1e-9 * (seed ^ threadIdx.x);                                      \
  double x0 = b+1, x1 = b+2, x2 = b+3, x3 = b+4, x4 = b+5, x5 = b+6, x6 = b+7, x7 = b+8; \
  for (int it = 0; it < ITER; ++it) {                                                \
    _Pragma("unroll")                                                                \
    for (int u = 0; u < 4; ++u) {                                                    \
      asm volatile(ASM : "+v"(x0) : "v"(b)); asm volatile(ASM : "+v"(x1) : "v"(b));  \
      asm volatile(ASM : "+v"(x2) : "v"(b)); asm volatile(ASM : "+v"(x3) : "v"(b));  \
      asm volatile(ASM : "+v"(x4) : "v"(b)); asm volatile(ASM : "+v"(x5) : "v"(b));  \
      asm volatile(ASM : "+v"(x6) : "v"(b)); asm volatile(ASM : "+v"(x7) : "v"(b));  \
    }                                                                                \
  }                                                                                  \
  double r = x0+x1+x2+x3+x4+x5+x6+x7;                                                \
  out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)__double2hiint(r);          \
}
KERN_F64(k_fma_f64, "v_fma_f64 %0, %0, %1, %1")
KERN_F64(k_mul_f64, "v_mul_f64 %0, %0, %1")
KERN_F64(k_rcp_f64, "v_rcp_f64 %0, %0")

// compiler-generated IEEE f64 division (8 independent divisions per iteration)
__global__ void __launch_bounds__(256) k_div_f64(uint32_t *out, uint32_t seed) {
  double b = 3.0 + 1e-9 * (seed ^ threadIdx.x);
  double x[8];
  for (int i = 0; i < 8; ++i) x[i] = 1.5 + i;
  for (int it = 0; it < ITER; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int i = 0; i < 8; ++i) { x[i] = x[i] / b; asm volatile("" : "+v"(x[i])); }
    }
  }
  double r = 0;
  for (int i = 0; i < 8; ++i) r += x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)__double2hiint(r);
}

// Streaming f64 store bandwidth: each thread writes consecutive 8B words, coalesced.
__global__ void __launch_bounds__(256) k_store_f64(double *dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = (double)i;
}
// Copy kernel (reads + writes), used as the known-size reference for traffic counters.
__global__ void __launch_bounds__(256) k_copy_f64(double *dst, const double *src, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

typedef void (*kfn)(uint32_t *, uint32_t);
struct Test { const char *name; kfn f; double ops_per_stmt; };

int main(int argc, char **argv) {
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  int cus = prop.multiProcessorCount;
  double clk_ghz = prop.clockRate / 1e6;
  printf("device %s gcn %s CUs %d clockRate %.3f GHz\n", prop.name, prop.gcnArchName, cus, clk_ghz);
  fflush(stdout);
  const int threads = 256;
  const int blocks = cus * 8;  // 8 WG of 4 waves each per CU -> 8 waves/SIMD
  uint32_t *out;
  CHECK(hipMalloc(&out, (size_t)blocks * threads * sizeof(uint32_t)));
  Test tests[] = {
    {"v_add_u32", k_add_u32, 1}, {"v_mul_lo_u32", k_mul_lo_u32, 1}, {"v_mul_hi_u32", k_mul_hi_u32, 1},
    {"v_mul_u32_u24", k_mul_u32_u24, 1}, {"v_mul_hi_u32_u24", k_mul_hi_u32_u24, 1},
    {"v_mad_u32_u24", k_mad_u32_u24, 1}, {"v_add3_u32", k_add3_u32, 1},
    {"v_alignbit_b32", k_alignbit, 1}, {"v_min_u32", k_min_u32, 1}, {"v_and_b32", k_and_b32, 1},
    {"v_cvt_f32_u32", k_cvt_f32_u32, 1},
    {"v_add_co+v_addc_co (2 insts)", k_addc, 2}, {"v_cmp+v_cndmask (2 insts)", k_cndmask, 2},
    {"v_mad_u64_u32", k_mad_u64_u32, 1}, {"v_mul_hi_u32+3*v_add (4 insts)", k_mulhi_plus3add, 4},
    {"v_fma_f64", k_fma_f64, 1}, {"v_mul_f64", k_mul_f64, 1}, {"v_rcp_f64", k_rcp_f64, 1},
    {"f64 '/' (per division)", k_div_f64, 1},
  };
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  for (auto &t : tests) {
    hipLaunchKernelGGL(t.f, dim3(blocks), dim3(threads), 0, 0, out, 1u);  // warm
    CHECK(hipDeviceSynchronize());
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      CHECK(hipEventRecord(e0));
      hipLaunchKernelGGL(t.f, dim3(blocks), dim3(threads), 0, 0, out, (uint32_t)rep + 2);
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) best = ms;
    }
    double stmts = (double)blocks * threads * ITER * 4 * 8;
    double lane_ops = stmts * t.ops_per_stmt;
    double per_cu_clk = lane_ops / (best * 1e-3) / cus / (clk_ghz * 1e9);
    printf("%-34s %9.3f ms  %8.3f Tlane-op/s  %6.2f lane-ops/CU/clk (stmt rate %6.2f /CU/clk)\n", t.name, best,
           lane_ops / (best * 1e-3) / 1e12, per_cu_clk, per_cu_clk / t.ops_per_stmt);
    fflush(stdout);
  }
  // store bandwidth
  size_t n = (size_t)1 << 31;  // 16 GiB of f64
  double *buf, *buf2;
  CHECK(hipMalloc(&buf, n * sizeof(double)));
  CHECK(hipMalloc(&buf2, n * sizeof(double)));
  for (int g : {cus * 4, cus * 8, cus * 16, cus * 32}) {
    hipLaunchKernelGGL(k_store_f64, dim3(g), dim3(256), 0, 0, buf, n);
    CHECK(hipDeviceSynchronize());
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      CHECK(hipEventRecord(e0));
      hipLaunchKernelGGL(k_store_f64, dim3(g), dim3(256), 0, 0, buf, n);
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) best = ms;
    }
    printf("store f64 grid %6d: %8.3f ms  %8.1f GB/s\n", g, best, n * 8.0 / (best * 1e-3) / 1e9);
    fflush(stdout);
  }
  {
    int g = cus * 16;
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      CHECK(hipEventRecord(e0));
      hipLaunchKernelGGL(k_copy_f64, dim3(g), dim3(256), 0, 0, buf2, buf, n);
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) best = ms;
    }
    printf("copy f64 16 GiB->16 GiB: %8.3f ms  %8.1f GB/s (read+write)\n", best, 2 * n * 8.0 / (best * 1e-3) / 1e9);
  }
  CHECK(hipFree(buf));
  CHECK(hipFree(buf2));
  CHECK(hipFree(out));
  printf("done\n");
  return 0;
}
