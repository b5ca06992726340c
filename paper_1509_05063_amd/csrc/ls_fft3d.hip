// In-place three-dimensional complex FFT of a dense n0 x n1 x n2 array in
// single precision: the zero-padded equivalent-source grid of the 3-D method
// (Sec. 4) transformed as one cube rather than per face-lattice set.  Three
// one-axis passes with the Stockham kernels of the face-lattice
// convolution: lines along the contiguous axis n2 (several per workgroup),
// 8-column tiles along n1 (16 for a 256-point axis), 16-column tiles along
// n0.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <vector>

#include "ls.h"
#include "ls_kernels.hpp"

struct ls_fft3d {
  int n[3] = {0, 0, 0};
  lsx::FftPlan plan[3]{};
  void* tw[3] = {nullptr, nullptr, nullptr};   // complex float exp(-2 pi i k / n) per axis
};

namespace {

bool smooth(int n) {
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

}  // namespace

extern "C" {

ls_status ls_fft3d_create(int n0, int n1, int n2, ls_fft3d** out) {
  if (!out) return LS_EINVAL;
  *out = nullptr;
  const int n[3] = {n0, n1, n2};
  for (int a = 0; a < 3; ++a)
    if (n[a] < 1 || !smooth(n[a])) return LS_EINVAL;
  // LDS per workgroup within 160 KB: lines of up to 2048 points; 8-column
  // tiles of n1 rows ((2 x 8 + 1) n1 values); 16-column tiles of n0 rows
  if (n2 > 2048 || 17LL * n1 * 8 > 160 * 1024 || 33LL * n0 * 8 > 160 * 1024 ||
      (int64_t)n0 * n1 * n2 > ((int64_t)1 << 31))
    return LS_EINVAL;
  if (lsx::set_fft_lds_limits(160 * 1024) != hipSuccess) return LS_EDEVICE;
  ls_fft3d* f = new ls_fft3d;
  for (int a = 0; a < 3; ++a) {
    f->n[a] = n[a];
    f->plan[a] = lsx::make_fft_plan(n[a]);
    std::vector<float> t(2 * (size_t)n[a]);
    for (int k = 0; k < n[a]; ++k) {
      const std::complex<double> w = std::polar(1.0, -2.0 * M_PI * (double)k / n[a]);
      t[2 * k] = (float)w.real();
      t[2 * k + 1] = (float)w.imag();
    }
    if (hipMalloc(&f->tw[a], 8 * (size_t)n[a]) != hipSuccess) {
      ls_fft3d_destroy(f);
      return LS_ENOMEM;
    }
    if (hipMemcpy(f->tw[a], t.data(), 8 * (size_t)n[a], hipMemcpyHostToDevice) != hipSuccess) {
      ls_fft3d_destroy(f);
      return LS_EDEVICE;
    }
  }
  *out = f;
  return LS_OK;
}

ls_status ls_fft3d_exec(ls_fft3d* f, void* data, int direction, void* stream) {
  if (!f || !data || (direction != 1 && direction != -1)) return LS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int n0 = f->n[0], n1 = f->n[1], n2 = f->n[2];
  const int64_t plane = (int64_t)n1 * n2;
  hipError_t e = lsx::launch_fft_lines(false, direction, data, data, f->tw[2], f->plan[2], n1, n2, plane, 0, n2,
                                       plane, 0, n0, 1, n2, n2, st);
  // 16-column tiles where the middle axis is two radix-16 passes (one LDS
  // buffer: 256 butterflies per pass for 256 threads), else 8
  const bool r16 = f->plan[1].npass == 2 && f->plan[1].radix[0] == 16 && f->plan[1].radix[1] == 16;
  if (e == hipSuccess)
    e = lsx::launch_fft_strided(false, direction, data, f->tw[1], f->plan[1], n2, r16 ? 16 : 8, plane, n0, n1, n1, 0,
                                1, st);
  if (e == hipSuccess)
    e = lsx::launch_fft_strided(false, direction, data, f->tw[0], f->plan[0], (int)plane, 16, 0, 1, n0, n0, 0, 1, st);
  return e == hipSuccess ? LS_OK : LS_EDEVICE;
}

void ls_fft3d_destroy(ls_fft3d* f) {
  if (!f) return;
  for (void* p : f->tw)
    if (p) (void)hipFree(p);
  delete f;
}

}  // extern "C"
