// Test and measurement entry points (include/peval_testing.h): the device
// modular arithmetic applied element by element, and the microbenchmark of
// the modular products and of the instructions they are built from.
#include "peval_testing.h"

#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "errors.hpp"
#include "modarith.hpp"
#include "peval_internal.hpp"

using namespace peval;

namespace {

struct ArithArgs {
  uint32_t op;
  Mod64 m64;
  Mod32 m32;
  ModF64 mf;
  uint64_t c;  // pseudo-Mersenne constant 2^k - p
  uint64_t count;
  const uint64_t *a, *b;
  uint64_t *out;
};

__device__ __forceinline__ double as_signed_double(uint64_t v) { return (double)(int64_t)v; }
__device__ __forceinline__ uint64_t from_signed_double(double v) { return (uint64_t)(int64_t)v; }

__global__ __launch_bounds__(256) void arith_test_kernel(ArithArgs x) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= x.count) return;
  const uint64_t a = x.a[i], b = x.b ? x.b[i] : 0;
  uint64_t r = 0;
  switch (x.op) {
    case PEVAL_TOP_MUL64: r = mul_mod(a, b, x.m64); break;
    case PEVAL_TOP_QUOT64: r = shoup_quot(a, x.m64); break;
    case PEVAL_TOP_SHOUP64: r = shoup_mul(a, b, shoup_quot(b, x.m64), x.m64.p); break;
    case PEVAL_TOP_REDUCE96: r = reduce96(a, (uint32_t)b, x.m64); break;
    case PEVAL_TOP_FOLD96: r = fold96(a, (uint32_t)b, x.m64); break;
    case PEVAL_TOP_POW64: r = pow_mod(a, b, x.m64); break;
    case PEVAL_TOP_SUM64: {
      W64::Sum s = W64::sum_zero();
      for (int k = 0; k < 16; ++k) W64::sum_add(s, x.a[16 * i + k]);
      r = W64::reduce(W64::stage(s, x.m64), x.m64);
      break;
    }
    case PEVAL_TOP_ALG2:
      r = from_signed_double(alg2_mul_signed(as_signed_double(a), (double)b, x.mf.p, x.mf.u));
      break;
    case PEVAL_TOP_FOLD: r = from_signed_double(fp_fold(as_signed_double(a), x.mf.p, x.mf.u)); break;
    case PEVAL_TOP_CANON_F64: r = WF64::reduce(WF64::Acc{as_signed_double(a)}, x.mf); break;
    case PEVAL_TOP_PM63: r = pm63_mul_lazy(a, b, x.c); break;
    case PEVAL_TOP_PM31: r = pm31_mul_lazy((uint32_t)a, (uint32_t)b, (uint32_t)x.c); break;
    case PEVAL_TOP_MUL32: r = mul_mod((uint32_t)a, (uint32_t)b, x.m32); break;
    case PEVAL_TOP_QUOT32: r = shoup_quot((uint32_t)a, x.m32); break;
    case PEVAL_TOP_SHOUP32: r = shoup_mul((uint32_t)a, (uint32_t)b, shoup_quot((uint32_t)b, x.m32), x.m32.p); break;
    case PEVAL_TOP_REDUCE64_32: r = reduce64(a, x.m32); break;
    case PEVAL_TOP_POW32: r = pow_mod((uint32_t)a, b, x.m32); break;
    case PEVAL_TOP_MONT32: r = mont_mul32((uint32_t)a, (uint32_t)b, x.m32.p, 0u - x.m32.pinv); break;
    case PEVAL_TOP_SUM32: {
      W32::Sum s = W32::sum_zero();
      for (int k = 0; k < 16; ++k) W32::sum_add(s, (uint32_t)x.a[16 * i + k]);
      r = W32::reduce(W32::stage(s, x.m32), x.m32);
      break;
    }
    default: break;
  }
  x.out[i] = r;
}

bool is_pm63(uint64_t p) { return p < (1ull << 63) && p > (1ull << 63) - (1ull << 20); }
bool is_pm31(uint64_t p) { return p < (1ull << 31) && p > (1ull << 31) - (1ull << 12); }

// Modulus range of each operation (0 = unknown op).
int op_class(uint32_t op) {
  switch (op) {
    case PEVAL_TOP_MUL64: case PEVAL_TOP_QUOT64: case PEVAL_TOP_SHOUP64: case PEVAL_TOP_REDUCE96:
    case PEVAL_TOP_POW64: case PEVAL_TOP_SUM64: case PEVAL_TOP_FOLD96: return 64;
    case PEVAL_TOP_ALG2: case PEVAL_TOP_FOLD: case PEVAL_TOP_CANON_F64: return 50;
    case PEVAL_TOP_PM63: return 63;
    case PEVAL_TOP_PM31: return 31;
    case PEVAL_TOP_MUL32: case PEVAL_TOP_QUOT32: case PEVAL_TOP_SHOUP32: case PEVAL_TOP_REDUCE64_32:
    case PEVAL_TOP_POW32: case PEVAL_TOP_SUM32: case PEVAL_TOP_MONT32: return 32;
    default: return 0;
  }
}

int check_modulus(int cls, uint64_t p) {
  const bool odd = p >= 3 && (p & 1);
  bool ok = false;
  switch (cls) {
    case 64: ok = odd && p < (1ull << 63); break;
    case 50: ok = odd && p >= (1ull << 31) && p < (1ull << 50); break;
    case 63: ok = is_pm63(p); break;
    case 31: ok = is_pm31(p); break;
    case 32: ok = odd && p < (1ull << 31); break;
    default: break;
  }
  return ok ? PEVAL_OK : fail(PEVAL_EINVAL, "modulus %llu outside the operation's range", (unsigned long long)p);
}

ModF64 make_modf64(uint64_t p) {
  ModF64 f;
  f.p = (double)p;
  f.u = 1.0 / (double)p;
  f.m = make_mod64(p);
  return f;
}

}  // namespace

extern "C" int peval_test_arith(uint32_t op, uint64_t p, uint64_t count, const uint64_t *dev_a,
                                const uint64_t *dev_b, uint64_t *dev_out, void *stream) {
  const int cls = op_class(op);
  if (!cls) return fail(PEVAL_EINVAL, "unknown operation %u", op);
  PEVAL_TRY(check_modulus(cls, p));
  if (count == 0) return PEVAL_OK;
  if (!dev_a || !dev_out) return fail(PEVAL_EINVAL, "null array");
  if (count > (1ull << 32)) return fail(PEVAL_EINVAL, "count too large");
  ArithArgs x;
  memset(&x, 0, sizeof x);
  x.op = op;
  x.m64 = make_mod64(p);
  if (p < (1ull << 31)) x.m32 = make_mod32((uint32_t)p);
  if (cls == 50) x.mf = make_modf64(p);
  x.c = cls == 63 ? (1ull << 63) - p : cls == 31 ? (1ull << 31) - p : 0;
  x.count = count;
  x.a = dev_a;
  x.b = dev_b;
  x.out = dev_out;
  arith_test_kernel<<<(unsigned)((count + 255) / 256), 256, 0, (hipStream_t)stream>>>(x);
  HIP_TRY(hipGetLastError());
  return PEVAL_OK;
}

// ---------------------------------------------------------------------------
// microbenchmark
// ---------------------------------------------------------------------------
namespace {

constexpr int kMbTable = 1024;  // multipliers per table (threads pick by index)

// Every thread: NCH running values with fixed multipliers; per iteration
// each value goes into the thread's sum and is multiplied by its
// multiplier; once per iteration the row's sum is staged and added into
// the thread's total, as in the evaluation kernel's loop.
template <class A, int NCH>
__global__ __launch_bounds__(256) void product_rate_kernel(typename A::M m, const typename A::T *wt,
                                                           const typename A::T *wqt, uint32_t iters,
                                                           uint64_t *sink) {
  using T = typename A::T;
  const uint32_t tid = blockIdx.x * 256 + threadIdx.x;
  T x[NCH], w[NCH], wq[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const uint32_t j = (tid * NCH + c) % kMbTable;
    w[c] = wt[j];
    wq[c] = wqt[j];
    x[c] = wt[(j + 1) % kMbTable];
  }
  typename A::Acc tot = A::zero();
  for (uint32_t it = 0; it < iters; ++it) {
    typename A::Sum acc = A::sum_zero();
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      A::sum_add(acc, x[c]);
      x[c] = A::mul_lazy(x[c], w[c], wq[c], m);
    }
    A::add_walk(tot, A::stage(acc, m), m);
  }
  sink[tid] = (uint64_t)A::reduce(tot, m);
}

#define MB_8(ins) ins(0) ins(1) ins(2) ins(3) ins(4) ins(5) ins(6) ins(7)

// Eight independent dependency chains of one instruction, sixteen
// instructions per iteration.
template <int KIND>
__global__ __launch_bounds__(256) void insn_rate_kernel(uint32_t iters, uint64_t *sink) {
  const uint32_t tid = blockIdx.x * 256 + threadIdx.x;
  const uint32_t k = tid | 1u;
  uint64_t res = 0;
  if constexpr (KIND == PEVAL_MB_ADD_U32 || KIND == PEVAL_MB_MUL_LO_U32 || KIND == PEVAL_MB_MUL_HI_U32) {
    uint32_t v0 = tid, v1 = tid + 1, v2 = tid + 2, v3 = tid + 3, v4 = tid + 4, v5 = tid + 5, v6 = tid + 6,
             v7 = tid + 7;
#define MB_LINE_ADD(i) "v_add_u32 %" #i ", %" #i ", %8\n\t"
#define MB_LINE_MULLO(i) "v_mul_lo_u32 %" #i ", %" #i ", %8\n\t"
#define MB_LINE_MULHI(i) "v_mul_hi_u32 %" #i ", %" #i ", %8\n\t"
    for (uint32_t it = 0; it < iters; ++it) {
      if constexpr (KIND == PEVAL_MB_ADD_U32)
        asm volatile(MB_8(MB_LINE_ADD) MB_8(MB_LINE_ADD)
                     : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(v3), "+v"(v4), "+v"(v5), "+v"(v6), "+v"(v7)
                     : "v"(k));
      else if constexpr (KIND == PEVAL_MB_MUL_LO_U32)
        asm volatile(MB_8(MB_LINE_MULLO) MB_8(MB_LINE_MULLO)
                     : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(v3), "+v"(v4), "+v"(v5), "+v"(v6), "+v"(v7)
                     : "v"(k));
      else
        asm volatile(MB_8(MB_LINE_MULHI) MB_8(MB_LINE_MULHI)
                     : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(v3), "+v"(v4), "+v"(v5), "+v"(v6), "+v"(v7)
                     : "v"(k));
    }
    res = (uint64_t)(v0 ^ v1 ^ v2 ^ v3 ^ v4 ^ v5 ^ v6 ^ v7);
  } else if constexpr (KIND == PEVAL_MB_MAD_U64_U32) {
    uint64_t v0 = tid, v1 = tid + 1, v2 = tid + 2, v3 = tid + 3, v4 = tid + 4, v5 = tid + 5, v6 = tid + 6,
             v7 = tid + 7, carry;
#define MB_LINE_MAD(i) "v_mad_u64_u32 %" #i ", %8, %9, %9, %" #i "\n\t"
    for (uint32_t it = 0; it < iters; ++it)
      asm volatile(MB_8(MB_LINE_MAD) MB_8(MB_LINE_MAD)
                   : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(v3), "+v"(v4), "+v"(v5), "+v"(v6), "+v"(v7), "=&s"(carry)
                   : "v"(k));
    res = v0 ^ v1 ^ v2 ^ v3 ^ v4 ^ v5 ^ v6 ^ v7;
  } else {
    double v0 = tid, v1 = tid + 1, v2 = tid + 2, v3 = tid + 3, v4 = tid + 4, v5 = tid + 5, v6 = tid + 6,
           v7 = tid + 7;
    const double a = 0.999, b = 1e-3;
#define MB_LINE_FMA(i) "v_fma_f64 %" #i ", %" #i ", %8, %9\n\t"
    for (uint32_t it = 0; it < iters; ++it)
      asm volatile(MB_8(MB_LINE_FMA) MB_8(MB_LINE_FMA)
                   : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(v3), "+v"(v4), "+v"(v5), "+v"(v6), "+v"(v7)
                   : "v"(a), "v"(b));
    res = (uint64_t)(v0 + v1 + v2 + v3 + v4 + v5 + v6 + v7);
  }
  sink[tid] = res;
}

// 64-bit xorshift for the multiplier tables.
uint64_t next_rand(uint64_t &s) {
  s ^= s << 13;
  s ^= s >> 7;
  s ^= s << 17;
  return s;
}

template <class T>
int upload_table(const std::vector<T> &v, void **d) {
  HIP_TRY(hipMalloc(d, v.size() * sizeof(T)));
  HIP_TRY(hipMemcpy(*d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return PEVAL_OK;
}

struct DevBufs {
  void *w = nullptr, *wq = nullptr, *sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~DevBufs() {
    if (w) (void)hipFree(w);
    if (wq) (void)hipFree(wq);
    if (sink) (void)hipFree(sink);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

typedef unsigned __int128 u128;

}  // namespace

extern "C" int peval_bench_product(uint32_t kind, uint64_t p, uint32_t iters, uint32_t blocks, double *ms,
                                   double *work) {
  if (!ms || !work) return fail(PEVAL_EINVAL, "null output");
  if (!blocks || blocks > (1u << 20) || !iters) return fail(PEVAL_EINVAL, "blocks and iters must be positive");
  const bool product = kind <= PEVAL_MB_PM31;
  const bool insn = kind >= PEVAL_MB_ADD_U32 && kind <= PEVAL_MB_FMA_F64;
  if (!product && !insn) return fail(PEVAL_EINVAL, "unknown kind %u", kind);
  if (product) {
    static const int cls[] = {64, 32, 50, 63, 31};
    PEVAL_TRY(check_modulus(cls[kind], p));
  }
  DevBufs d;
  const uint64_t threads = (uint64_t)blocks * 256;
  HIP_TRY(hipMalloc(&d.sink, threads * 8));
  HIP_TRY(hipEventCreate(&d.e0));
  HIP_TRY(hipEventCreate(&d.e1));
  uint64_t seed = 0x9e3779b97f4a7c15ull ^ p;
  std::vector<uint64_t> w64(kMbTable), wq64(kMbTable);
  std::vector<uint32_t> w32(kMbTable), wq32(kMbTable);
  std::vector<double> wf(kMbTable);
  for (int j = 0; j < kMbTable; ++j) {
    const uint64_t w = product ? next_rand(seed) % p : 0;
    w64[j] = w;
    wq64[j] = product ? (uint64_t)(((u128)w << 64) / p) : 0;
    w32[j] = (uint32_t)w;
    wq32[j] = product && p < (1ull << 32) ? (uint32_t)(((uint64_t)w << 32) / p) : 0;
    wf[j] = (double)w;
  }
  int nch = 16;
  auto launch = [&]() -> int {
    switch (kind) {
      case PEVAL_MB_SHOUP64:
        product_rate_kernel<W64, 16><<<blocks, 256>>>(make_mod64(p), (const uint64_t *)d.w,
                                                      (const uint64_t *)d.wq, iters, (uint64_t *)d.sink);
        break;
      case PEVAL_MB_SHOUP32:
        product_rate_kernel<W32, 16><<<blocks, 256>>>(make_mod32((uint32_t)p), (const uint32_t *)d.w,
                                                      (const uint32_t *)d.wq, iters, (uint64_t *)d.sink);
        break;
      case PEVAL_MB_FP64:
        nch = 8;
        product_rate_kernel<WF64, 8><<<blocks, 256>>>(make_modf64(p), (const double *)d.w, (const double *)d.wq,
                                                      iters, (uint64_t *)d.sink);
        break;
      case PEVAL_MB_PM63:
        product_rate_kernel<W64PM, 16><<<blocks, 256>>>(ModPM64{p, (1ull << 63) - p, make_mod64(p)},
                                                        (const uint64_t *)d.w, (const uint64_t *)d.wq, iters,
                                                        (uint64_t *)d.sink);
        break;
      case PEVAL_MB_PM31:
        product_rate_kernel<W32PM, 16><<<blocks, 256>>>(
            ModPM32{(uint32_t)p, (uint32_t)((1ull << 31) - p), make_mod32((uint32_t)p)}, (const uint32_t *)d.w,
            (const uint32_t *)d.wq, iters, (uint64_t *)d.sink);
        break;
      case PEVAL_MB_ADD_U32: insn_rate_kernel<PEVAL_MB_ADD_U32><<<blocks, 256>>>(iters, (uint64_t *)d.sink); break;
      case PEVAL_MB_MUL_LO_U32:
        insn_rate_kernel<PEVAL_MB_MUL_LO_U32><<<blocks, 256>>>(iters, (uint64_t *)d.sink);
        break;
      case PEVAL_MB_MUL_HI_U32:
        insn_rate_kernel<PEVAL_MB_MUL_HI_U32><<<blocks, 256>>>(iters, (uint64_t *)d.sink);
        break;
      case PEVAL_MB_MAD_U64_U32:
        insn_rate_kernel<PEVAL_MB_MAD_U64_U32><<<blocks, 256>>>(iters, (uint64_t *)d.sink);
        break;
      default: insn_rate_kernel<PEVAL_MB_FMA_F64><<<blocks, 256>>>(iters, (uint64_t *)d.sink); break;
    }
    HIP_TRY(hipGetLastError());
    return PEVAL_OK;
  };
  if (product) {
    if (kind == PEVAL_MB_SHOUP32 || kind == PEVAL_MB_PM31) {
      PEVAL_TRY(upload_table(w32, &d.w));
      PEVAL_TRY(upload_table(wq32, &d.wq));
    } else if (kind == PEVAL_MB_FP64) {
      PEVAL_TRY(upload_table(wf, &d.w));
      PEVAL_TRY(upload_table(wf, &d.wq));
    } else {
      PEVAL_TRY(upload_table(w64, &d.w));
      PEVAL_TRY(upload_table(wq64, &d.wq));
    }
  }
  PEVAL_TRY(launch());  // warm-up (code object load, clocks)
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipEventRecord(d.e0, 0));
  PEVAL_TRY(launch());
  HIP_TRY(hipEventRecord(d.e1, 0));
  HIP_TRY(hipEventSynchronize(d.e1));
  float t = 0;
  HIP_TRY(hipEventElapsedTime(&t, d.e0, d.e1));
  *ms = t;
  *work = product ? (double)threads * iters * nch : (double)threads * iters * 16;
  return PEVAL_OK;
}
