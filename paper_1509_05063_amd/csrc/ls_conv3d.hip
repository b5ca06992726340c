// The FFT convolution step of the three-dimensional method (Sec. 3.2,
// equiv-conv-loc): per source set, the monopole and dipole strengths on the
// set's face lattice are convolved with the free-space Helmholtz Green's
// function G(r) = exp(i kappa r) / (4 pi r) and its derivative along the
// set's normal axis, by zero-padded FFTs.  The lattice of a set is indexed
// [a][b][c] = (normal, tangential, tangential) with spacings hn, ht, ht;
// every set of a cubic cell lattice has the same dimensions, and in its own
// (normal, tangential, tangential) frame the same kernels, so one pair of
// spectra serves all sets.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <vector>

#include "ls.h"
#include "ls_kernels.hpp"
#include "ls_setup.hpp"

struct ls_conv3d {
  int na = 0, nb = 0, nc = 0, nsets = 0;
  int Pa = 0, Pb = 0, Pc = 0;
  lsx::FftPlan pa{}, pb{}, pc{};
  void *twa = nullptr, *twb = nullptr, *twc = nullptr;   // complex float twiddles per axis
  void* khat = nullptr;                                  // [2 kinds][Pa][Pb][Pc] complex float spectra
  size_t resident = 0;
};

namespace {

using cd = std::complex<double>;

// ws[s][k][a][b][c] (padded strides) <- sig[s][k][a][b][c] (compact), the
// na x nb x nc corner only: the transforms read no element outside it
__global__ void k_pad3(const float2* __restrict__ sig, float2* __restrict__ ws, int na, int nb, int nc, int Pb,
                       int Pc, int64_t P, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t per = (int64_t)na * nb * nc;
  const int64_t arr = i / per, rest = i % per;
  const int a = (int)(rest / ((int64_t)nb * nc)), b = (int)(rest / nc % nb), c = (int)(rest % nc);
  ws[arr * P + ((int64_t)a * Pb + b) * Pc + c] = sig[i];
}

// field[s][a][b][c] <- ws[s][0][a][b][c]
__global__ void k_unpad3(const float2* __restrict__ ws, float2* __restrict__ field, int na, int nb, int nc, int Pb,
                         int Pc, int64_t P, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t per = (int64_t)na * nb * nc;
  const int64_t s = i / per, rest = i % per;
  const int a = (int)(rest / ((int64_t)nb * nc)), b = (int)(rest / nc % nb), c = (int)(rest % nc);
  field[i] = ws[(2 * s) * P + ((int64_t)a * Pb + b) * Pc + c];
}

std::vector<cd> twiddles(int n) {
  std::vector<cd> t(n);
  for (int k = 0; k < n; ++k) t[k] = std::polar(1.0, -2.0 * M_PI * (double)k / n);
  return t;
}

ls_status upload(const void* src, size_t bytes, void** dst, size_t* resident) {
  *dst = nullptr;
  if (hipMalloc(dst, bytes) != hipSuccess) return LS_ENOMEM;
  if (resident) *resident += bytes;
  if (hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return LS_EDEVICE;
  return LS_OK;
}

std::vector<float> to_float(const std::vector<cd>& v) {
  std::vector<float> f(2 * v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    f[2 * i] = (float)v[i].real();
    f[2 * i + 1] = (float)v[i].imag();
  }
  return f;
}

// full forward transform (all three axes, no padding skipped) of nz double
// arrays spaced zstride apart: the kernel spectra
hipError_t forward3_double(void* data, const lsx::FftPlan& pa, const lsx::FftPlan& pb, const lsx::FftPlan& pc,
                           const void* twa, const void* twb, const void* twc, int Pa, int Pb, int Pc, int64_t zstride,
                           int nz) {
  const int64_t plane = (int64_t)Pb * Pc;
  hipError_t e;
  if ((e = lsx::launch_fft_lines(true, 1, data, twc, pc, Pc, Pb, Pc, Pc, plane, Pa, zstride, nz, 0))) return e;
  if ((e = lsx::launch_fft_strided(true, 1, data, twb, pb, Pc, 4, plane, Pa, Pb, Pb, zstride, nz, 0))) return e;
  return lsx::launch_fft_strided(true, 1, data, twa, pa, (int)plane, 16, 0, 1, Pa, Pa, zstride, nz, 0);
}

}  // namespace

extern "C" {

ls_status ls_conv3d_create(int na, int nb, int nc, double hn, double ht, double kappa, int nsets, ls_conv3d** out) {
  if (!out) return LS_EINVAL;
  *out = nullptr;
  if (na < 1 || nb < 1 || nc < 1 || nsets < 1 || !(hn > 0) || !(ht > 0) || !(kappa > 0)) return LS_EINVAL;
  ls_conv3d* c = new ls_conv3d;
  c->na = na;
  c->nb = nb;
  c->nc = nc;
  c->nsets = nsets;
  c->Pa = lsx::next_smooth(2 * na - 1);
  c->Pb = lsx::next_smooth(2 * nb - 1);
  c->Pc = lsx::next_smooth(2 * nc - 1);
  const int Pa = c->Pa, Pb = c->Pb, Pc = c->Pc;
  const int64_t P = (int64_t)Pa * Pb * Pc;
  // line transforms stage two lines of the axis length in LDS; strided ones
  // two tiles of it (8 columns along the second axis, 4 in double; along
  // the normal axis 16 columns of both kinds, or 16 double columns for the
  // spectra); all within the default 64 KB
  if (Pc > 2048 || (int64_t)Pb * Pc > (int64_t)1 << 30 || 2LL * Pb * 8 * 16 > 64 * 1024 ||
      2LL * Pa * 16 * 16 > 64 * 1024) {
    delete c;
    return LS_EINVAL;
  }
  c->pa = lsx::make_fft_plan(Pa);
  c->pb = lsx::make_fft_plan(Pb);
  c->pc = lsx::make_fft_plan(Pc);
  auto cleanup = [&](ls_status s) {
    ls_conv3d_destroy(c);
    return s;
  };
  ls_status s;
  std::vector<cd> ta = twiddles(Pa), tb = twiddles(Pb), tc = twiddles(Pc);
  if ((s = upload(to_float(ta).data(), 8 * (size_t)Pa, &c->twa, &c->resident))) return cleanup(s);
  if ((s = upload(to_float(tb).data(), 8 * (size_t)Pb, &c->twb, &c->resident))) return cleanup(s);
  if ((s = upload(to_float(tc).data(), 8 * (size_t)Pc, &c->twc, &c->resident))) return cleanup(s);
  // kernel lattices in double: offsets (da hn, db ht, dc ht) wrapped into
  // the padded box, K(0) = 0, scaled by 1 / (Pa Pb Pc) for the inverse
  std::vector<cd> ker((size_t)(2 * P), cd(0.0, 0.0));
  const double scale = 1.0 / (double)P;
#pragma omp parallel for schedule(static)
  for (int ia = 0; ia < Pa; ++ia) {
    const int da = ia < na ? ia : ia - Pa;
    if (da <= -na || da >= na) continue;
    for (int ib = 0; ib < Pb; ++ib) {
      const int db = ib < nb ? ib : ib - Pb;
      if (db <= -nb || db >= nb) continue;
      for (int ic = 0; ic < Pc; ++ic) {
        const int dc = ic < nc ? ic : ic - Pc;
        if (dc <= -nc || dc >= nc) continue;
        if (da == 0 && db == 0 && dc == 0) continue;
        const double dn = da * hn, d1 = db * ht, d2 = dc * ht;
        const double r = std::sqrt(dn * dn + d1 * d1 + d2 * d2);
        const cd g = std::exp(cd(0.0, kappa * r)) / (4.0 * M_PI * r);
        const cd gp = g * cd(-1.0, kappa * r) / r;        // dG/dr
        const size_t o = ((size_t)ia * Pb + ib) * Pc + ic;
        ker[o] = g * scale;
        ker[(size_t)P + o] = -gp * (dn / r) * scale;      // d/dy_n G(|x - y|), x - y = offset
      }
    }
  }
  void *kd = nullptr, *twa64 = nullptr, *twb64 = nullptr, *twc64 = nullptr;
  auto free_tmp = [&]() {
    for (void* p : {kd, twa64, twb64, twc64})
      if (p) (void)hipFree(p);
  };
  if ((s = upload(ker.data(), 16 * (size_t)(2 * P), &kd, nullptr)) || (s = upload(ta.data(), 16 * (size_t)Pa, &twa64, nullptr)) ||
      (s = upload(tb.data(), 16 * (size_t)Pb, &twb64, nullptr)) || (s = upload(tc.data(), 16 * (size_t)Pc, &twc64, nullptr))) {
    free_tmp();
    return cleanup(s);
  }
  // spectra: full forward transforms in double (no padding skipped: the
  // wrapped offsets fill the box)
  hipError_t e = forward3_double(kd, c->pa, c->pb, c->pc, twa64, twb64, twc64, Pa, Pb, Pc, P, 2);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(ker.data(), kd, 16 * (size_t)(2 * P), hipMemcpyDeviceToHost);
  free_tmp();
  if (e != hipSuccess) return cleanup(LS_EDEVICE);
  if ((s = upload(to_float(ker).data(), 8 * (size_t)(2 * P), &c->khat, &c->resident))) return cleanup(s);
  *out = c;
  return LS_OK;
}

ls_status ls_conv3d_info(const ls_conv3d* c, int* padded, size_t* ws_bytes, size_t* resident_bytes) {
  if (!c) return LS_EINVAL;
  if (padded) {
    padded[0] = c->Pa;
    padded[1] = c->Pb;
    padded[2] = c->Pc;
  }
  if (ws_bytes) *ws_bytes = (size_t)c->nsets * 2 * (size_t)c->Pa * c->Pb * c->Pc * 8;
  if (resident_bytes) *resident_bytes = c->resident;
  return LS_OK;
}

ls_status ls_conv3d_apply(ls_conv3d* c, const void* sigma, void* field, void* ws, size_t ws_bytes, void* stream) {
  if (!c || !sigma || !field || !ws) return LS_EINVAL;
  const int64_t P = (int64_t)c->Pa * c->Pb * c->Pc;
  if (ws_bytes < (size_t)c->nsets * 2 * (size_t)P * 8) return LS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int64_t nin = (int64_t)c->nsets * 2 * c->na * c->nb * c->nc, nout = nin / 2;
  hipLaunchKernelGGL(k_pad3, dim3((unsigned)((nin + 255) / 256)), dim3(256), 0, st, (const float2*)sigma,
                     (float2*)ws, c->na, c->nb, c->nc, c->Pb, c->Pc, P, nin);
  hipError_t e = hipGetLastError();
  const int64_t plane = (int64_t)c->Pb * c->Pc;
  const int na = c->na, nb = c->nb, nc = c->nc, Pb = c->Pb, Pc = c->Pc;
  // forward along c and b for both kinds of every set
  if (e == hipSuccess)
    e = lsx::launch_fft_lines(false, 1, ws, c->twc, c->pc, Pc, nb, nc, Pc, plane, na, P, 2 * c->nsets, st);
  if (e == hipSuccess)
    e = lsx::launch_fft_strided(false, 1, ws, c->twb, c->pb, Pc, 8, plane, na, nb, Pb, P, 2 * c->nsets, st);
  // along a: forward, spectral product, inverse in one pass; rows a < na of
  // kind 0 hold the result
  if (e == hipSuccess)
    e = lsx::launch_fft_conv_strided(ws, c->twa, c->khat, c->pa, (int)plane, 16, P, na, c->nsets, st);
  // inverse along b and c of kind 0 of every set
  if (e == hipSuccess)
    e = lsx::launch_fft_strided(false, -1, ws, c->twb, c->pb, Pc, 8, plane, na, Pb, nb, 2 * P, c->nsets, st);
  if (e == hipSuccess)
    e = lsx::launch_fft_lines(false, -1, ws, c->twc, c->pc, Pc, nb, Pc, nc, plane, na, 2 * P, c->nsets, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_unpad3, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, st, (const float2*)ws,
                       (float2*)field, c->na, c->nb, c->nc, c->Pb, c->Pc, P, nout);
    e = hipGetLastError();
  }
  return e == hipSuccess ? LS_OK : LS_EDEVICE;
}

void ls_conv3d_destroy(ls_conv3d* c) {
  if (!c) return;
  for (void* p : {c->twa, c->twb, c->twc, c->khat})
    if (p) (void)hipFree(p);
  delete c;
}

}  // extern "C"
