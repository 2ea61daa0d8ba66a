// Coefficients back from the images (Zippel's sparse interpolation with a
// known support, paper Section 2.1).  Kernels in interp_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>

#include "errors.hpp"
#include "interp_kernels.hpp"
#include "peval.h"
#include "peval_internal.hpp"

using namespace peval;

namespace {

__global__ void interp_status_reset(int32_t *status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) status[0] = 0;
}

template <class A>
const typename A::M &mod_for(const peval_poly *h);
template <>
const Mod64 &mod_for<W64>(const peval_poly *h) { return h->m64; }
template <>
const Mod32 &mod_for<W32>(const peval_poly *h) { return h->m32; }

static void free_interp_arrays(peval_poly *h) {
  uint32_t **arrays[] = {&h->d_order, &h->d_gorder, &h->d_task_group, &h->d_task_first};
  for (uint32_t **a : arrays) {
    if (*a) (void)hipFree(*a);
    *a = nullptr;
  }
  for (auto &lvl : h->d_mt)
    for (uint32_t *&a : lvl) {
      if (a) (void)hipFree(a);
      a = nullptr;
    }
}

static int interp_setup_once(peval_poly *h);

// Device copies of the sort order and group structure (first complete call
// only; a setup that failed half way is undone and tried again next time).
int interp_setup(peval_poly *h) {
  if (h->interp_ready) return PEVAL_OK;
  free_interp_arrays(h);
  const int rc = interp_setup_once(h);
  if (rc != PEVAL_OK) {
    free_interp_arrays(h);
    return rc;
  }
  h->interp_ready = true;
  return PEVAL_OK;
}

static int interp_setup_once(peval_poly *h) {
  std::vector<uint32_t> off32(h->G + 1), gord(h->G);
  for (uint64_t g = 0; g <= h->G; ++g) off32[g] = (uint32_t)h->grp_off[g];
  std::iota(gord.begin(), gord.end(), 0u);
  std::stable_sort(gord.begin(), gord.end(), [&](uint32_t x, uint32_t y) {
    return h->grp_off[x + 1] - h->grp_off[x] > h->grp_off[y + 1] - h->grp_off[y];
  });
  HIP_TRY(hipMalloc((void **)&h->d_order, std::max<size_t>(h->order.size(), 1) * 4));
  if (!h->d_grp_off32) {  // (uploaded at create for small polynomials)
    uint32_t *d = nullptr;
    HIP_TRY(hipMalloc((void **)&d, off32.size() * 4));
    if (hipMemcpy(d, off32.data(), off32.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return fail(PEVAL_EDEVICE, "group offsets upload");
    }
    h->d_grp_off32 = d;
  }
  HIP_TRY(hipMalloc((void **)&h->d_gorder, std::max<size_t>(gord.size(), 1) * 4));
  HIP_TRY(hipMemcpy(h->d_order, h->order.data(), h->order.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_gorder, gord.data(), gord.size() * 4, hipMemcpyHostToDevice));
  // solve tasks: one wave per 64 consecutive terms of one group
  std::vector<uint32_t> tg, tf;
  for (uint64_t g = 0; g < h->G; ++g)
    for (uint64_t j = 0; j < h->grp_off[g + 1] - h->grp_off[g]; j += 64) {
      tg.push_back((uint32_t)g);
      tf.push_back((uint32_t)j);
    }
  h->ntasks = tg.size();
  // few groups: Q as 4 or 8 sub-products per group (one wave or block
  // each), merged pairwise in chip-wide levels, so that more than G waves
  // share the work (two sub-products for 256-2047 groups measured no faster:
  // the merge costs what the shorter products save)
  uint64_t mx = 0;
  for (uint64_t g = 0; g < h->G; ++g) mx = std::max<uint64_t>(mx, h->grp_off[g + 1] - h->grp_off[g]);
  h->interp_H = (mx < 256 || h->G >= 256) ? 1 : (h->G < 128 ? 8 : 4);
  for (uint32_t lvl = 0, Hl = h->interp_H; Hl > 1; ++lvl, Hl /= 2) {
    std::vector<uint32_t> mg, mp, mf;
    for (uint64_t g = 0; g < h->G; ++g) {
      const uint64_t m = h->grp_off[g + 1] - h->grp_off[g];
      for (uint32_t j = 0; j < Hl / 2; ++j) {
        const uint64_t deg = ((2 * j + 2) * m) / Hl - ((2 * j) * m) / Hl;  // degree of the product
        for (uint64_t k = 0; k <= deg; k += 64) {
          mg.push_back((uint32_t)g);
          mp.push_back(j);
          mf.push_back((uint32_t)k);
        }
      }
    }
    h->mt_n[lvl] = mg.size();
    for (int q = 0; q < 3; ++q) {
      const std::vector<uint32_t> &src = q == 0 ? mg : q == 1 ? mp : mf;
      HIP_TRY(hipMalloc((void **)&h->d_mt[lvl][q], std::max<size_t>(src.size(), 1) * 4));
      HIP_TRY(hipMemcpy(h->d_mt[lvl][q], src.data(), src.size() * 4, hipMemcpyHostToDevice));
    }
  }
  HIP_TRY(hipMalloc((void **)&h->d_task_group, std::max<size_t>(tg.size(), 1) * 4));
  HIP_TRY(hipMalloc((void **)&h->d_task_first, std::max<size_t>(tf.size(), 1) * 4));
  HIP_TRY(hipMemcpy(h->d_task_group, tg.data(), tg.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_task_first, tf.data(), tf.size() * 4, hipMemcpyHostToDevice));
  return PEVAL_OK;
}

uint64_t largest_group(const peval_poly *h) {
  uint64_t mx = 0;
  for (uint64_t g = 0; g < h->G; ++g) mx = std::max<uint64_t>(mx, h->grp_off[g + 1] - h->grp_off[g]);
  return mx;
}

template <class A>
int interp_impl(peval_poly *h, const BetaArg &beta, const void *images, uint64_t *out, int32_t *status,
                hipStream_t st) {
  using T_ = typename A::T;
  const auto &m = mod_for<A>(h);
  const size_t w = sizeof(T_);
  const uint32_t ntail = h->n - 2;
  PEVAL_TRY(interp_setup(h));
  PEVAL_TRY(ensure(h->tabval, (size_t)std::max<uint32_t>(h->tab_total, 1) * w, h));
  PEVAL_TRY(ensure(h->tabquot, (size_t)std::max<uint32_t>(h->tab_total, 1) * w, h));
  // m, m', c, c', b, Q' (s each), Q (s + G), and two buffers of parts with
  // quotients that the merge levels alternate between (s + 8G, twice each)
  PEVAL_TRY(ensure(h->iscr, ((size_t)11 * h->s + 33 * h->G) * w, h));
  interp_status_reset<<<1, 64, 0, st>>>(status);
  HIP_TRY(hipGetLastError());
  if (ntail) {
    ProfScope ps(st, 0);
    power_table_kernel<A><<<(h->tab_total + 255) / 256, 256, 0, st>>>(beta, h->tab, ntail, h->tab_total,
                                                                      (T_ *)h->tabval.ptr, (T_ *)h->tabquot.ptr, m);
    HIP_TRY(hipGetLastError());
  }
  InterpArgs<A> a;
  T_ *scr = (T_ *)h->iscr.ptr;
  a.images = (const T_ *)images;
  a.tval = (const T_ *)h->tabval.ptr;
  a.tquot = (const T_ *)h->tabquot.ptr;
  a.to = h->tab;
  a.exps = h->d_exps;
  a.grp_off = h->d_grp_off32;
  a.gorder = h->d_gorder;
  a.order = h->d_order;
  a.mval = scr;
  a.mquot = scr + h->s;
  a.cval = scr + 2 * h->s;
  a.cquot = scr + 3 * h->s;
  a.bval = scr + 4 * h->s;
  a.dval = scr + 5 * h->s;
  a.qval = scr + 6 * h->s;
  T_ *lv0 = a.qval + h->s + h->G;           // parts (values, quotients)
  T_ *lv0q = lv0 + h->s + 8 * h->G;
  T_ *lv1 = lv0q + h->s + 8 * h->G;         // the next level, then back to lv0
  T_ *lv1q = lv1 + h->s + 8 * h->G;
  a.part_val = lv0;
  a.part_quot = lv0q;
  a.H = h->interp_H;
  a.task_group = h->d_task_group;
  a.task_first = h->d_task_first;
  a.ntasks = h->ntasks;
  a.out = out;
  a.status = status;
  a.s = h->s;
  a.G = h->G;
  a.ntail = ntail;
  a.m = m;
  a.fp64 = (sizeof(T_) == 8 && h->arith == 1) ? 1u : 0u;  // the handle's product resolves to FP64
  a.mf = h->mf;
  {
    ProfScope ps(st, 1);
    interp_prep_kernel<A><<<(unsigned)((h->s + 255) / 256), 256, 0, st>>>(a);
    HIP_TRY(hipGetLastError());
  }
  {
    // parts below 1024 roots: one wave each, in registers; larger ones one
    // block each in LDS (256 threads up to 8 * 256 - 1 roots, else 1024)
    const uint64_t mx = largest_group(h);
    const uint64_t part = (mx + a.H - 1) / a.H + 1;
    const size_t shmem = (part + 1) * w;
    const unsigned blocks = (unsigned)(h->G * a.H);
    ProfScope ps(st, 2);
    if (part - 1 < (uint64_t)kWaveGroupSlots * 64) {  // every part has fewer than 1024 roots
      const uint32_t nparts = (uint32_t)(h->G * a.H);
      interp_wave_group_kernel<A, kWaveGroupSlots><<<(nparts + 3) / 4, 256, 0, st>>>(a, nparts);
    } else if (part >= (uint64_t)kInterpPer * 256) {
      interp_group_kernel<A, 1024><<<blocks, 1024, shmem, st>>>(a);
    } else {
      interp_group_kernel<A, 256><<<blocks, 256, shmem, st>>>(a);
    }
    HIP_TRY(hipGetLastError());
    T_ *in_v = lv0, *in_q = lv0q;
    for (uint32_t lvl = 0, Hl = a.H; Hl > 1; ++lvl, Hl /= 2) {
      const bool last = Hl == 2;
      T_ *nv = (in_v == lv0) ? lv1 : lv0, *nq = (in_v == lv0) ? lv1q : lv0q;
      T_ *out_v = last ? a.qval : nv, *out_q = last ? nullptr : nq;
      interp_merge_kernel<A><<<(unsigned)((h->mt_n[lvl] + 3) / 4), 256, 0, st>>>(
          a, in_v, in_q, out_v, out_q, Hl, h->d_mt[lvl][0], h->d_mt[lvl][1], h->d_mt[lvl][2], h->mt_n[lvl]);
      HIP_TRY(hipGetLastError());
      in_v = out_v;
      in_q = out_q;
    }
    interp_bcoef_kernel<A><<<(unsigned)((h->ntasks + 3) / 4), 256, 0, st>>>(a);
    HIP_TRY(hipGetLastError());
  }
  {
    ProfScope ps(st, 3);
    interp_solve_kernel<A><<<(unsigned)((h->ntasks + 3) / 4), 256, 0, st>>>(a);
    HIP_TRY(hipGetLastError());
  }
  return PEVAL_OK;
}

int check_interp(peval_poly *h, const uint64_t *beta, uint32_t T, const void *images, const void *out,
                 BetaArg *ba) {
  if (!h) return fail(PEVAL_EINVAL, "null handle");
  if (h->n > 2 && !beta) return fail(PEVAL_EINVAL, "null beta");
  if (h->s && (!images || !out)) return fail(PEVAL_EINVAL, "null images or output");
  const uint64_t mx = largest_group(h);
  if (T < mx) return fail(PEVAL_EINVAL, "T = %u images, the largest group has %llu terms", T, (unsigned long long)mx);
  if (mx > kInterpMaxGroup)
    return fail(PEVAL_EUNSUPPORTED, "a group of %llu terms (at most %u)", (unsigned long long)mx, kInterpMaxGroup);
  memset(ba, 0, sizeof *ba);
  for (uint32_t k = 0; k + 2 < h->n; ++k) ba->b[k] = beta[k] % h->p;
  return PEVAL_OK;
}

int interp_locked(peval_poly *h, const BetaArg &ba, const void *images, uint64_t *out, int32_t *status,
                  hipStream_t st) {
  HIP_TRY(hipSetDevice(h->device));
  if (h->have_done) HIP_TRY(hipStreamWaitEvent(st, h->done, 0));
  int rc = (h->w == 4) ? interp_impl<W32>(h, ba, images, out, status, st)
                       : interp_impl<W64>(h, ba, images, out, status, st);
  if (rc != PEVAL_OK) return rc;
  HIP_TRY(hipEventRecord(h->done, st));
  h->have_done = true;
  return PEVAL_OK;
}

}  // namespace

extern "C" int peval_interpolate_async(peval_poly *h, const uint64_t *beta, uint32_t T, const void *dev_images,
                                       uint64_t *dev_coeffs, int32_t *dev_status, void *stream) {
  BetaArg ba;
  PEVAL_TRY(check_interp(h, beta, T, dev_images, dev_coeffs, &ba));
  if (!dev_status) return fail(PEVAL_EINVAL, "null status");
  if (h->s == 0) return PEVAL_OK;
  std::lock_guard<std::mutex> lk(h->mu);
  return interp_locked(h, ba, dev_images, dev_coeffs, dev_status, (hipStream_t)stream);
}

extern "C" int peval_interpolate(peval_poly *h, const uint64_t *beta, uint32_t T, const void *images,
                                 uint64_t *coeffs) {
  BetaArg ba;
  PEVAL_TRY(check_interp(h, beta, T, images, coeffs, &ba));
  if (h->s == 0) return PEVAL_OK;
  std::lock_guard<std::mutex> lk(h->mu);
  // only the first (largest group) rows of the images are read
  const uint64_t rows = largest_group(h);
  const size_t ibytes = ((size_t)rows * h->G * h->w + 255) / 256 * 256;
  const size_t obytes = (size_t)h->s * 8;
  PEVAL_TRY(ensure(h->ptsbuf, ibytes + obytes + 256, h));
  unsigned char *base = (unsigned char *)h->ptsbuf.ptr;
  int32_t *dstatus = (int32_t *)(base + ibytes + obytes);
  HIP_TRY(hipMemcpyAsync(base, images, (size_t)rows * h->G * h->w, hipMemcpyHostToDevice, h->stream));
  PEVAL_TRY(interp_locked(h, ba, base, (uint64_t *)(base + ibytes), dstatus, h->stream));
  int32_t status = 0;
  HIP_TRY(hipMemcpyAsync(coeffs, base + ibytes, obytes, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(&status, dstatus, sizeof status, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (status) return fail(PEVAL_ESINGULAR, "a group's system is singular (equal or zero monomial values, or p not prime)");
  return PEVAL_OK;
}
