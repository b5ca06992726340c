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
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ls.h"
#include "ls_kernels.hpp"
#include "ls_setup.hpp"

struct ls_conv3d {
  int na = 0, nb = 0, nc = 0, nsets = 0;
  int Pa = 0, Pb = 0, Pc = 0;
  lsx::FftPlan pa{}, pb{}, pc{};
  void *twa = nullptr, *twb = nullptr, *twc = nullptr;   // complex float twiddles per axis
  void* khs = nullptr;   // [2 kinds][Pa/2+1][Pb/2+1][Pc/2+1] complex float: one octant of the spectra
  size_t resident = 0;
  // schedule: columns and threads per workgroup of the fused normal-axis
  // pass, columns per workgroup along the second axis, and the skew: values
  // of padding after each normal-axis plane of the workspace (planes Pb Pc +
  // skew apart, so that the rows one workgroup of the normal-axis pass
  // reads do not all fall at one power-of-two stride) (ls_conv3d_autotune)
  int tc_a = 16, nth_a = 256, tc_b = 8, skew = 0;
  int64_t pstride() const { return (int64_t)Pb * Pc + skew; }
  int64_t vol() const { return (int64_t)Pa * pstride(); }
};

namespace {
constexpr int kMaxSkew = 512;   // complex values (4 KB)
size_t ws_need(const ls_conv3d* c) { return (size_t)c->nsets * 2 * (size_t)c->Pa * ((size_t)c->Pb * c->Pc + kMaxSkew) * 8; }
}  // namespace

namespace {

using cd = std::complex<double>;

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
  if ((e = lsx::launch_fft_lines(true, 1, data, data, twc, pc, Pb, Pc, plane, zstride, Pc, plane, zstride, Pa, nz, Pc,
                                 Pc, 0)))
    return e;
  if ((e = lsx::launch_fft_strided(true, 1, data, twb, pb, Pc, 4, plane, Pa, Pb, Pb, zstride, nz, 0))) return e;
  return lsx::launch_fft_strided(true, 1, data, twa, pa, (int)plane, 16, 0, 1, Pa, Pa, zstride, nz, 0);
}

}  // namespace

extern "C" {

ls_status ls_conv3d_create(int na, int nb, int nc, double hn, double ht, double kappa, int nsets, ls_conv3d** out) {
  if (!out) return LS_EINVAL;
  *out = nullptr;
  if (na < 1 || nb < 1 || nc < 1 || nsets < 1 || nsets > 1024 || !(hn > 0) || !(ht > 0) || !(kappa > 0))
    return LS_EINVAL;
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
  // LDS per workgroup (the FFT kernels are allowed 160 KB; every transform
  // also stages the axis' twiddles): line transforms two buffers of n (L +
  // 1) values with L <= 2048 / n lines (1024 / n in double); strided ones
  // two tiles of the axis length (8 columns along the second axis, 4 in
  // double: Pb <= 512; along the normal axis 16 columns of both kinds, or
  // 16 double columns for the spectra: Pa <= 128)
  if (Pc > 2048 || Pb > 512 || Pa > 128 || (int64_t)Pb * Pc > (int64_t)1 << 30) {
    delete c;
    return LS_EINVAL;
  }
  if (lsx::set_fft_lds_limits(160 * 1024) != hipSuccess) {
    delete c;
    return LS_EDEVICE;
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
  // keep the octant 0 <= k <= P/2 per axis (the spectra are even per axis,
  // the dipole's odd along the normal one: the apply mirrors the rest)
  const int ha = Pa / 2 + 1, hb = Pb / 2 + 1, hc = Pc / 2 + 1;
  const size_t hsz = (size_t)ha * hb * hc;
  std::vector<cd> oct(2 * hsz);
  for (int k = 0; k < 2; ++k)
    for (int ia = 0; ia < ha; ++ia)
      for (int ib = 0; ib < hb; ++ib)
        for (int ic = 0; ic < hc; ++ic)
          oct[k * hsz + ((size_t)ia * hb + ib) * hc + ic] = ker[(size_t)k * P + ((size_t)ia * Pb + ib) * Pc + ic];
  if ((s = upload(to_float(oct).data(), 8 * 2 * hsz, &c->khs, &c->resident))) return cleanup(s);
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
  if (ws_bytes) *ws_bytes = ws_need(c);
  if (resident_bytes) *resident_bytes = c->resident;
  return LS_OK;
}

}  // extern "C"

namespace {

hipError_t pass_b(ls_conv3d* c, void* ws, int dir, hipStream_t st) {
  const int64_t ps = c->pstride(), V = c->vol();
  if (dir > 0)
    return lsx::launch_fft_strided(false, 1, ws, c->twb, c->pb, c->Pc, c->tc_b, ps, c->na, c->nb, c->Pb, V,
                                   2 * c->nsets, st);
  return lsx::launch_fft_strided(false, -1, ws, c->twb, c->pb, c->Pc, c->tc_b, ps, c->na, c->Pb, c->nb, 2 * V,
                                 c->nsets, st);
}

hipError_t pass_a(ls_conv3d* c, void* ws, hipStream_t st) {
  return lsx::launch_fft_conv_octant(ws, c->twa, c->khs, c->pa, c->Pb, c->Pc, c->tc_a, c->nth_a, c->pstride(),
                                     c->vol(), c->na, c->nsets, st);
}

}  // namespace

extern "C" {

ls_status ls_conv3d_apply(ls_conv3d* c, const void* sigma, void* field, void* ws, size_t ws_bytes, void* stream) {
  if (!c || !sigma || !field || !ws) return LS_EINVAL;
  if (ws_bytes < ws_need(c)) return LS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int na = c->na, nb = c->nb, nc = c->nc, Pc = c->Pc, ns = c->nsets;
  const int64_t plane = c->pstride(), P = c->vol(), cplane = (int64_t)nb * nc, cvol = (int64_t)na * cplane;
  // forward along c, straight from the compact strengths (rows b < nb of
  // planes a < na), then along b (planes a < na), both kinds of every set
  hipError_t e = lsx::launch_fft_lines(false, 1, sigma, ws, c->twc, c->pc, nb, nc, cplane, cvol, Pc, plane, P, na,
                                       2 * ns, nc, Pc, st);
  if (e == hipSuccess) e = pass_b(c, ws, 1, st);
  // along a: forward, spectral product, inverse in one pass; rows a < na of
  // kind 0 hold the result
  if (e == hipSuccess) e = pass_a(c, ws, st);
  // inverse along b, then along c straight into the compact field, kind 0
  if (e == hipSuccess) e = pass_b(c, ws, -1, st);
  if (e == hipSuccess)
    e = lsx::launch_fft_lines(false, -1, ws, field, c->twc, c->pc, nb, Pc, plane, 2 * P, nc, cplane, cvol, na, ns, Pc,
                              nc, st);
  return e == hipSuccess ? LS_OK : LS_EDEVICE;
}

ls_status ls_conv3d_autotune(ls_conv3d* c, void* ws, size_t ws_bytes, void* stream, int* schedule) {
  if (!c || !ws) return LS_EINVAL;
  if (ws_bytes < ws_need(c)) return LS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const bool logc = std::getenv("LS_TUNE_LOG") != nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return LS_EDEVICE;
  }
  ls_status rc = LS_OK;
  // average of 3 launches after one untimed one; the transforms run on
  // whatever the workspace holds (cleared first: finite values)
  auto timed = [&](auto&& launch, double* ms) -> bool {
    if (launch() != hipSuccess || hipEventRecord(e0, st) != hipSuccess) return false;
    for (int r = 0; r < 3; ++r)
      if (launch() != hipSuccess) return false;
    float t = 0;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess)
      return false;
    *ms = t / 3.0;
    return true;
  };
  if (hipMemsetAsync(ws, 0, ws_need(c), st) != hipSuccess) rc = LS_EDEVICE;
  // plane skew, timed over all passes but the line transforms
  int best_skew = c->skew;
  double bsk = 1e30;
  for (int sk : {0, 32, 64, kMaxSkew}) {
    if (rc) break;
    c->skew = sk;
    double t;
    if (!timed(
            [&] {
              hipError_t e = pass_b(c, ws, 1, st);
              if (e == hipSuccess) e = pass_a(c, ws, st);
              return e == hipSuccess ? pass_b(c, ws, -1, st) : e;
            },
            &t)) {
      rc = LS_EDEVICE;
      break;
    }
    if (logc) std::fprintf(stderr, "ls_conv3d_autotune plane skew %d: %.4f ms\n", sk, t);
    if (t < bsk) {
      bsk = t;
      best_skew = sk;
    }
  }
  c->skew = best_skew;
  // fused normal-axis pass: tile width and threads (LDS within 160 KB)
  int best_tc = c->tc_a, best_nth = c->nth_a;
  double best = 1e30;
  for (int tc : {4, 8, 16, 32, 64}) {
    if ((4 * (size_t)tc + 1) * c->Pa * 8 > 160 * 1024) break;
    for (int nth : {256, 512}) {
      if (rc) break;
      c->tc_a = tc;
      c->nth_a = nth;
      double t;
      if (!timed([&] { return pass_a(c, ws, st); }, &t)) {
        rc = LS_EDEVICE;
        break;
      }
      if (logc) std::fprintf(stderr, "ls_conv3d_autotune normal-axis tile %d threads %d: %.4f ms\n", tc, nth, t);
      if (t < best) {
        best = t;
        best_tc = tc;
        best_nth = nth;
      }
    }
  }
  c->tc_a = best_tc;
  c->nth_a = best_nth;
  // second-axis passes (forward and inverse): tile width
  int best_b = c->tc_b;
  best = 1e30;
  for (int tc : {4, 8, 16}) {
    if (rc || (2 * (size_t)tc + 1) * c->Pb * 8 > 160 * 1024) break;
    c->tc_b = tc;
    double t;
    if (!timed(
            [&] {
              hipError_t e = pass_b(c, ws, 1, st);
              return e == hipSuccess ? pass_b(c, ws, -1, st) : e;
            },
            &t)) {
      rc = LS_EDEVICE;
      break;
    }
    if (logc) std::fprintf(stderr, "ls_conv3d_autotune second-axis tile %d: %.4f ms\n", tc, t);
    if (t < best) {
      best = t;
      best_b = tc;
    }
  }
  c->tc_b = best_b;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == LS_OK && schedule) {
    schedule[0] = c->tc_a;
    schedule[1] = c->nth_a;
    schedule[2] = c->tc_b;
    schedule[3] = c->skew;
  }
  return rc;
}

ls_status ls_conv3d_set_schedule(ls_conv3d* c, const int* schedule) {
  if (!c || !schedule) return LS_EINVAL;
  const int ta = schedule[0], na = schedule[1], tb = schedule[2], sk = schedule[3];
  if (ta < 1 || ta > 64 || (na != 256 && na != 512) || tb < 1 || tb > 16 || sk < 0 || sk > kMaxSkew ||
      (4 * (size_t)ta + 1) * c->Pa * 8 > 160 * 1024 || (2 * (size_t)tb + 1) * c->Pb * 8 > 160 * 1024)
    return LS_EINVAL;
  c->tc_a = ta;
  c->nth_a = na;
  c->tc_b = tb;
  c->skew = sk;
  return LS_OK;
}

void ls_conv3d_destroy(ls_conv3d* c) {
  if (!c) return;
  for (void* p : {c->twa, c->twb, c->twc, c->khs})
    if (p) (void)hipFree(p);
  delete c;
}

}  // extern "C"
