// Measurement harness for the HBM traffic of the batched complex product kernel
// (not part of libnegf.so).  It compiles the kernel's own source and launches,
// at b = 512 and a given batch, one streaming kernel of known size (reads and
// writes 1 GiB: the calibration of the memory counters) and then the five
// operand forms the RGF sweeps use on the full-tile path with three real
// products per complex one and 64 x 64 eight-wave tiles:
//   NN, NN with C as input, CN, NC, CC with C as input
// (two warm-up and `reps` timed launches each).  Run it under
//   rocprofv3 --pmc FETCH_SIZE ...   and   rocprofv3 --pmc WRITE_SIZE ...
// and reduce with `python -m paper_2602_03438_amd.profsummary --traffic`.
//
//   gemm_traffic [batch=128] [reps=2]
#include "../csrc/gemm.hip"

#include <cstdio>
#include <cstdlib>
#include <vector>

namespace negf {
// the library's launch-time profiling hooks are not linked into this program
void prof_begin(int, hipStream_t) {}
void prof_end(int, hipStream_t, double, double) {}
}  // namespace negf

using namespace negf;

#define CHK(x)                                                                              \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) {                                                                 \
      fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);        \
      exit(1);                                                                              \
    }                                                                                       \
  } while (0)

// dst = -src over n4 float4 values: reads and writes 16 n4 bytes
__global__ void elementwise_copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst, long n4) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n4; i += (long)gridDim.x * blockDim.x)
    dst[i] = make_float4(-src[i].x, -src[i].y, -src[i].z, -src[i].w);
}

template <int OA, int OB>
void launch(KArgs ka, int reps, const char* label) {
  typedef Cfg64w8 CF;
  ka.tiles_m = ka.M / CF::BM;
  ka.tiles_n = ka.N / CF::BN;
  const dim3 grid((unsigned)(ka.tiles_m * ka.tiles_n * ka.batch)), block(CF::NT);
  for (int r = 0; r < 2 + reps; ++r)
    hipLaunchKernelGGL((zgemm_kernel<double, OA, OB, CF, 0, true, true>), grid, block, 0, 0, ka);
  CHK(hipGetLastError());
  CHK(hipDeviceSynchronize());
  printf("%s: %d launches of %d products\n", label, 2 + reps, ka.batch);
  fflush(stdout);
}

int main(int argc, char** argv) {
  const int n = 512;
  const int batch = argc > 1 ? atoi(argv[1]) : 128;
  const int reps = argc > 2 ? atoi(argv[2]) : 2;
  if (batch < 1 || batch > 512 || reps < 1 || reps > 100) {
    fprintf(stderr, "usage: gemm_traffic [batch 1..512] [reps 1..100]\n");
    return 2;
  }
  // calibration: 1 GiB read, 1 GiB written
  const long n4 = (1L << 30) / 16;
  float4 *cs, *cd;
  CHK(hipMalloc(&cs, n4 * 16));
  CHK(hipMalloc(&cd, n4 * 16));
  CHK(hipMemset(cs, 0, n4 * 16));
  hipLaunchKernelGGL(elementwise_copy_kernel, dim3(4096), dim3(256), 0, 0, cs, cd, n4);
  CHK(hipGetLastError());
  CHK(hipDeviceSynchronize());
  CHK(hipFree(cs));
  CHK(hipFree(cd));
  printf("calibration copy of 1024 MiB done\n");

  const size_t el = (size_t)n * n * batch;
  std::vector<double2> h(el);
  unsigned s = 12345u;
  for (size_t i = 0; i < el; ++i) {
    s = s * 1664525u + 1013904223u;
    const double re = (double)(s >> 8) / 16777216.0 - 0.5;
    s = s * 1664525u + 1013904223u;
    const double im = (double)(s >> 8) / 16777216.0 - 0.5;
    h[i] = make_double2(re, im);
  }
  double2 *A, *B, *C;
  CHK(hipMalloc(&A, el * 16));
  CHK(hipMalloc(&B, el * 16));
  CHK(hipMalloc(&C, el * 16));
  CHK(hipMemcpy(A, h.data(), el * 16, hipMemcpyHostToDevice));
  CHK(hipMemcpy(B, h.data(), el * 16, hipMemcpyHostToDevice));
  CHK(hipMemcpy(C, h.data(), el * 16, hipMemcpyHostToDevice));

  KArgs k{};
  k.M = k.N = k.K = n;
  k.batch = batch;
  k.A = A; k.lda = n; k.sA = (long)n * n;
  k.B = B; k.ldb = n; k.sB = (long)n * n;
  k.Cin = C; k.ldci = n; k.sCi = (long)n * n;
  k.C = C; k.ldc = n; k.sC = (long)n * n;
  k.alpha = make_double2(1.0, 0.0);
  k.beta = make_double2(0.0, 0.0);
  k.active = nullptr; k.xcd_remap = 1; k.upper = 0; k.kmask = nullptr; k.kmask_op = 0;
  KArgs kc = k;
  kc.beta = make_double2(1.0, 0.0);
  launch<OP_N, OP_N>(k, reps, "NN");
  launch<OP_N, OP_N>(kc, reps, "NN, C as input");
  launch<OP_C, OP_N>(k, reps, "CN");
  launch<OP_N, OP_C>(k, reps, "NC");
  launch<OP_C, OP_C>(kc, reps, "CC, C as input");
  CHK(hipFree(A));
  CHK(hipFree(B));
  CHK(hipFree(C));
  printf("done\n");
  return 0;
}
