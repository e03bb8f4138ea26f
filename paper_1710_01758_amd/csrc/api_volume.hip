// C ABI of the 3D extension: a context per volume, the system operator, the
// 3D circulant preconditioner and PCG.  The 3D transforms run as the 2D
// row / column passes over the planes of a volume plus a column pass of
// length p over the volume viewed as one [p][m n] array.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "fft.hpp"
#include "internal.hpp"
#include "pics.h"

using namespace pics;

struct pics3d_ctx {
  hipStream_t stream = nullptr;
  pics3d_desc d{};
  long long V = 0;
  const float2* sens = nullptr;
  const uint8_t* mask = nullptr;
  void* block = nullptr;
  float2 *tw, *coil, *r, *z, *p, *q, *t;
  float *kraw, *kinv, *P;
  double *part, *scal;
  int* bad;
  int* flag_host = nullptr;  // pinned
  double* scal_host = nullptr;  // pinned
  // slice tables viewing the coil buffer / one volume as planes and as [p][m n]
  SliceDev *planes_coil, *planes_vol, *z_coil, *z_vol;
  int* idx;  // 0, 1, 2, ... (grid.y -> slice)
  bool built = false;
  bool xconst = false;  // mask constant along x: the operator's three-pass (z, y) path
  int xchunk_opt = 0;    // PICS3D_OPT_XCHUNK (0: automatic)
  char err[256] = {0};
};

namespace {

int fail3(pics3d_ctx* c, int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(c->err, sizeof c->err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK3(ctx, expr)                                                                           \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return fail3(ctx, PICS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

Ws ws3(const pics3d_ctx* c, const SliceDev* sl) {
  Ws w{};
  w.sl = sl;
  w.group = c->idx;
  w.tw = c->tw;
  return w;
}

Launch launch3(const pics3d_ctx* c, int m, int n, int count) {
  Launch L;
  L.stream = c->stream;
  L.m = m;
  L.n = n;
  L.count = count;
  L.group = c->idx;
  return L;
}

// In-place (through t) unnormalised 3D transform of `count` volumes at buf:
// rows, columns and z of every volume.  inverse: e^{+i}.
int fft3(pics3d_ctx* c, float2* buf, int count, int inverse, float2* scratch) {
  const int p = c->d.p, m = c->d.m, n = c->d.n;
  const SliceDev* planes = count > 1 ? c->planes_coil : c->planes_vol;
  const SliceDev* zs = count > 1 ? c->z_coil : c->z_vol;
  HIPCHK3(c, launch_row_fft(launch3(c, m, n, count * p), ws3(c, planes), inverse, 0, buf, scratch));
  HIPCHK3(c, launch_col_fft(launch3(c, m, n, count * p), ws3(c, planes), inverse, scratch, buf));
  HIPCHK3(c, launch_col_fft(launch3(c, p, m * n, count), ws3(c, zs), inverse, buf, scratch));
  HIPCHK3(c, hipMemcpyAsync(buf, scratch, sizeof(float2) * c->V * count, hipMemcpyDeviceToDevice, c->stream));
  return PICS_OK;
}

// x-chunk width of the x-constant operator: the option if set, else the
// widest chunk (a multiple of the m axis' column tile dividing n) whose coil
// workspace [nc][p][m][X] fits kVolChunkBytes, half the 256 MiB last-level
// cache (the chunk's coil maps, read by the first and the last pass, take
// the other half)
constexpr long long kVolChunkBytes = 128ll << 20;
int xchunk(const pics3d_ctx* c) {
  if (c->xchunk_opt > 0) return c->xchunk_opt;
  const int T = col_tile(c->d.m), n = c->d.n;
  const long long per_col = (long long)c->d.ncoils * c->d.p * c->d.m * (long long)sizeof(float2);
  int best = T;
  for (int X = T; X <= n; X += T)
    if (n % X == 0 && per_col * X <= kVolChunkBytes) best = X;
  return best;
}

bool xchunk_ok(const pics3d_ctx* c, int X) {
  const int T = col_tile(c->d.m);
  return X >= T && X <= c->d.n && X % T == 0 && c->d.n % X == 0;
}

int apply3(pics3d_ctx* c, const float2* x, float2* y) {
  const int nc = c->d.ncoils;
  if (c->xconst) {
    // F^H R F = (F_zy^H R_zy F_zy) (x) I_x: transforms along y and z only,
    // chunk by chunk along x through one chunk-sized workspace
    const int p = c->d.p, m = c->d.m, n = c->d.n, X = xchunk(c);
    const float scale = (float)(1.0 / ((double)p * m));
    for (int x0 = 0; x0 < n; x0 += X) {
      HIPCHK3(c, launch3_col_sp(c->stream, c->sens, x, c->coil, c->tw, nc, p, m, n, x0, X));
      HIPCHK3(c, launch3_col_z(c->stream, c->coil, c->mask, c->tw, nc, p, m, n, x0, X, scale));
      HIPCHK3(c, launch3_col_acc(c->stream, c->sens, c->coil, x, y, c->tw, nc, p, m, n, (float)c->d.mu,
                                 (float)c->d.lambda, (float)c->d.gamma, 1, x0, X));
    }
    return PICS_OK;
  }
  HIPCHK3(c, launch3_coil_mul(c->stream, c->sens, x, c->coil, nc, c->V));
  // the coil transforms use the second half of the coil workspace as scratch
  float2* scratch = c->coil + (long long)nc * c->V;
  int rc = fft3(c, c->coil, nc, 0, scratch);
  if (rc) return rc;
  HIPCHK3(c, launch3_mask_scale(c->stream, c->coil, c->mask, nc, c->V, (float)(1.0 / (double)c->V)));
  rc = fft3(c, c->coil, nc, 1, scratch);
  if (rc) return rc;
  HIPCHK3(c, launch3_accumulate(c->stream, c->sens, c->coil, x, y, nc, c->d.p, c->d.m, c->d.n, (float)c->d.mu,
                                (float)c->d.lambda, (float)c->d.gamma, 1));
  return PICS_OK;
}

int minv3(pics3d_ctx* c, const float2* r, float2* z) {
  HIPCHK3(c, hipMemcpyAsync(z, r, sizeof(float2) * c->V, hipMemcpyDeviceToDevice, c->stream));
  int rc = fft3(c, z, 1, 0, c->t);
  if (rc) return rc;
  HIPCHK3(c, launch3_scale(c->stream, z, c->kinv, c->V));
  return fft3(c, z, 1, 1, c->t);
}

bool size_ok(int s) { return fft_size_supported(s); }

}  // namespace

extern "C" {

int pics3d_create(pics3d_ctx** out, const pics3d_desc* d, const void* sens, const uint8_t* mask, void* stream) {
  if (!out) return PICS_ERR_INVALID;
  *out = nullptr;
  if (!d || !sens || !mask) return PICS_ERR_INVALID;
  if (d->p <= 0 || d->m <= 0 || d->n <= 0 || d->ncoils < 1 || d->ncoils > 4096) return PICS_ERR_INVALID;
  if (!(std::isfinite(d->mu) && d->mu >= 0) || !(std::isfinite(d->lambda) && d->lambda >= 0) ||
      !(std::isfinite(d->gamma) && d->gamma >= 0))
    return PICS_ERR_INVALID;
  if (!size_ok(d->p) || !size_ok(d->m) || !size_ok(d->n)) return PICS_ERR_UNSUPPORTED;
  pics3d_ctx* c = new pics3d_ctx();
  c->d = *d;
  c->stream = (hipStream_t)stream;
  c->sens = (const float2*)sens;
  c->mask = mask;
  const int p = d->p, m = d->m, n = d->n, nc = d->ncoils;
  c->V = (long long)p * m * n;
  const int nplanes = nc * p;
  std::vector<std::pair<void**, size_t>> plan;
  auto add = [&](void** ptr, size_t bytes) { plan.push_back({ptr, (bytes + 255) / 256 * 256}); };
  add((void**)&c->tw, sizeof(float2) * kTwiddleTotal);
  add((void**)&c->coil, sizeof(float2) * 2 * nc * c->V);  // coil volumes + transform scratch
  for (float2** b : {&c->r, &c->z, &c->p, &c->q, &c->t}) add((void**)b, sizeof(float2) * c->V);
  for (float** b : {&c->kraw, &c->kinv, &c->P}) add((void**)b, sizeof(float) * c->V);
  add((void**)&c->part, sizeof(double) * 4 * kVolDotBlocks);
  add((void**)&c->scal, sizeof(double) * 8);
  add((void**)&c->bad, sizeof(int));
  add((void**)&c->planes_coil, sizeof(SliceDev) * nplanes);
  add((void**)&c->planes_vol, sizeof(SliceDev) * p);
  add((void**)&c->z_coil, sizeof(SliceDev) * nc);
  add((void**)&c->z_vol, sizeof(SliceDev));
  add((void**)&c->idx, sizeof(int) * nplanes);
  size_t total = 0;
  for (auto& e : plan) total += e.second;
  if (hipMalloc(&c->block, total) != hipSuccess) {
    delete c;
    return PICS_ERR_HIP;
  }
  size_t off = 0;
  for (auto& e : plan) {
    *e.first = (char*)c->block + off;
    off += e.second;
  }
  std::vector<float2> tw(kTwiddleTotal);
  fill_twiddles(tw.data());
  auto view = [&](int count, int mm, int nn, long long stride) {
    std::vector<SliceDev> v(count);
    for (int i = 0; i < count; ++i) {
      SliceDev s{};
      s.m = mm;
      s.n = nn;
      s.nc = 1;
      s.img = stride * i;
      v[i] = s;
    }
    return v;
  };
  const auto pc = view(nplanes, m, n, (long long)m * n), pv = view(p, m, n, (long long)m * n);
  const auto zc = view(nc, p, m * n, c->V), zv = view(1, p, m * n, c->V);
  std::vector<int> idx(nplanes);
  for (int i = 0; i < nplanes; ++i) idx[i] = i;
  bool ok = hipMemcpy(c->tw, tw.data(), sizeof(float2) * kTwiddleTotal, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->planes_coil, pc.data(), sizeof(SliceDev) * nplanes, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->planes_vol, pv.data(), sizeof(SliceDev) * p, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->z_coil, zc.data(), sizeof(SliceDev) * nc, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->z_vol, zv.data(), sizeof(SliceDev), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->idx, idx.data(), sizeof(int) * nplanes, hipMemcpyHostToDevice) == hipSuccess &&
            hipHostMalloc((void**)&c->flag_host, sizeof(int)) == hipSuccess &&
            hipHostMalloc((void**)&c->scal_host, sizeof(double) * 8) == hipSuccess;
  // is the mask constant along x?  (then the operator skips the x transforms)
  ok = ok && hipMemsetAsync(c->bad, 0, sizeof(int), c->stream) == hipSuccess &&
       launch3_xconst(c->stream, mask, (long long)p * m, n, c->bad) == hipSuccess &&
       hipMemcpyAsync(c->flag_host, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
       hipStreamSynchronize(c->stream) == hipSuccess;
  if (ok) c->xconst = *c->flag_host == 0;
  if (!ok) {
    if (c->flag_host) (void)hipHostFree(c->flag_host);
    if (c->scal_host) (void)hipHostFree(c->scal_host);
    (void)hipFree(c->block);
    delete c;
    return PICS_ERR_HIP;
  }
  *out = c;
  return PICS_OK;
}

int pics3d_destroy(pics3d_ctx* c) {
  if (!c) return PICS_ERR_INVALID;
  // best-effort release: errors are ignored on the way out
  (void)hipStreamSynchronize(c->stream);
  (void)hipHostFree(c->flag_host);
  (void)hipHostFree(c->scal_host);
  (void)hipFree(c->block);
  delete c;
  return PICS_OK;
}

const char* pics3d_last_error(const pics3d_ctx* c) { return c ? c->err : "null context"; }

int pics3d_set_option(pics3d_ctx* c, int32_t option, int32_t value) {
  if (!c) return PICS_ERR_INVALID;
  if (option != PICS3D_OPT_XCHUNK) return fail3(c, PICS_ERR_INVALID, "set_option: unknown option %d", option);
  if (value != 0 && !xchunk_ok(c, value))
    return fail3(c, PICS_ERR_INVALID, "set_option: x chunk %d must be a multiple of %d dividing %d", value,
                 col_tile(c->d.m), c->d.n);
  c->xchunk_opt = value;
  return PICS_OK;
}

int pics3d_get_option(const pics3d_ctx* c, int32_t option, int32_t* value) {
  if (!c || !value) return PICS_ERR_INVALID;
  if (option != PICS3D_OPT_XCHUNK) return PICS_ERR_INVALID;
  *value = c->xconst ? xchunk(c) : 0;
  return PICS_OK;
}

int pics3d_apply_A(pics3d_ctx* c, const void* x, void* y) {
  if (!c) return PICS_ERR_INVALID;
  if (!x || !y || x == y) return fail3(c, PICS_ERR_INVALID, "apply_A: null or aliased buffers");
  return apply3(c, (const float2*)x, (float2*)y);
}

int pics3d_build_preconditioner(pics3d_ctx* c, int32_t kind, float* khat_out) {
  if (!c) return PICS_ERR_INVALID;
  if (kind == PICS_PRECOND_NONE) {
    c->built = false;
    return PICS_OK;
  }
  if (kind != PICS_PRECOND_CIRCULANT) return fail3(c, PICS_ERR_UNSUPPORTED, "3D: none or circulant only");
  const int nc = c->d.ncoils;
  // P = sum_c |DFT(s_c)|^2 through the coil workspace
  HIPCHK3(c, hipMemcpyAsync(c->coil, c->sens, sizeof(float2) * nc * c->V, hipMemcpyDeviceToDevice, c->stream));
  int rc = fft3(c, c->coil, nc, 0, c->coil + (long long)nc * c->V);
  if (rc) return rc;
  HIPCHK3(c, launch3_power(c->stream, c->coil, c->P, nc, c->V));
  // k_c = IDFT(DFT(r) conj(DFT(P))) / N^3
  HIPCHK3(c, launch3_corr_prep(c->stream, c->mask, c->P, c->r, c->z, c->V));
  if ((rc = fft3(c, c->r, 1, 0, c->t))) return rc;
  if ((rc = fft3(c, c->z, 1, 0, c->t))) return rc;
  HIPCHK3(c, launch3_corr_mul(c->stream, c->r, c->z, c->V));
  if ((rc = fft3(c, c->r, 1, 1, c->t))) return rc;
  HIPCHK3(c, hipMemsetAsync(c->bad, 0, sizeof(int), c->stream));
  HIPCHK3(c, launch3_build_k(c->stream, c->r, c->kraw, c->kinv, c->bad, c->d.p, c->d.m, c->d.n, c->d.mu,
                             c->d.lambda, c->d.gamma));
  HIPCHK3(c, hipMemcpyAsync(c->flag_host, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  if (khat_out)
    HIPCHK3(c, hipMemcpyAsync(khat_out, c->kraw, sizeof(float) * c->V, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK3(c, hipStreamSynchronize(c->stream));
  if (*c->flag_host) return fail3(c, PICS_ERR_NOT_POSITIVE, "3D circulant spectrum not positive");
  c->built = true;
  return PICS_OK;
}

int pics3d_rhs(pics3d_ctx* c, const void* kspace, void* b) {
  if (!c) return PICS_ERR_INVALID;
  if (!kspace || !b) return fail3(c, PICS_ERR_INVALID, "rhs: null buffer");
  const int nc = c->d.ncoils;
  HIPCHK3(c, hipMemcpyAsync(c->coil, kspace, sizeof(float2) * nc * c->V, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK3(c, launch3_mask_scale(c->stream, c->coil, c->mask, nc, c->V, (float)(1.0 / std::sqrt((double)c->V))));
  int rc = fft3(c, c->coil, nc, 1, c->coil + (long long)nc * c->V);
  if (rc) return rc;
  HIPCHK3(c, hipMemsetAsync(c->q, 0, sizeof(float2) * c->V, c->stream));
  HIPCHK3(c, launch3_accumulate(c->stream, c->sens, c->coil, c->q, (float2*)b, nc, c->d.p, c->d.m, c->d.n,
                                (float)c->d.mu, 0.f, 0.f, 1));
  return PICS_OK;
}

int pics3d_apply_Minv(pics3d_ctx* c, const void* r, void* z) {
  if (!c) return PICS_ERR_INVALID;
  if (!r || !z || r == z) return fail3(c, PICS_ERR_INVALID, "apply_Minv: null or aliased buffers");
  if (!c->built) return fail3(c, PICS_ERR_STATE, "apply_Minv: no circulant build");
  return minv3(c, (const float2*)r, (float2*)z);
}

// Preconditioned CG (Saad, Alg. 9.1) as in pcg_solve; alpha and beta are
// formed on the device from FP64 inner products; the host reads ||r||^2 and
// ||b||^2 after every iteration for the stop test.
int pics3d_pcg_solve(pics3d_ctx* c, const void* bv, void* xv, double tol, int32_t maxit, int32_t* iters_out,
                     double* relres_out) {
  if (!c) return PICS_ERR_INVALID;
  if (!bv || !xv || bv == xv) return fail3(c, PICS_ERR_INVALID, "pcg_solve: null or aliased buffers");
  if (!(tol >= 0.0) || maxit < 0) return fail3(c, PICS_ERR_INVALID, "pcg_solve: tol / maxit");
  const float2* b = (const float2*)bv;
  float2* x = (float2*)xv;
  const long long V = c->V;
  enum { RHO0 = 0, RHO1 = 1, SIG = 2, RR = 3, BB = 4 };
  auto z_of = [&](float2* out) -> int {  // z = M^{-1} r
    if (c->built) return minv3(c, c->r, out);
    HIPCHK3(c, hipMemcpyAsync(out, c->r, sizeof(float2) * V, hipMemcpyDeviceToDevice, c->stream));
    return PICS_OK;
  };
  auto read_rr = [&](double* rr, double* bb) -> int {
    HIPCHK3(c, hipMemcpyAsync(c->scal_host, c->scal, sizeof(double) * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    *rr = c->scal_host[RR];
    *bb = c->scal_host[BB];
    return PICS_OK;
  };
  int rc = apply3(c, x, c->q);
  if (rc) return rc;
  HIPCHK3(c, launch3_residual(c->stream, b, c->q, c->r, V));
  HIPCHK3(c, launch3_dot(c->stream, b, b, V, c->part, 0, c->scal, BB));
  HIPCHK3(c, launch3_dot(c->stream, c->r, c->r, V, c->part, 1, c->scal, RR));
  double rr, bb;
  if ((rc = read_rr(&rr, &bb))) return rc;
  int it = 0;
  int status = 0;
  if (bb == 0.0) {
    HIPCHK3(c, hipMemsetAsync(x, 0, sizeof(float2) * V, c->stream));
    status = 1;
  } else if (rr <= tol * tol * bb) {
    status = 1;
  } else {
    if ((rc = z_of(c->z))) return rc;
    HIPCHK3(c, launch3_dot(c->stream, c->r, c->z, V, c->part, 2, c->scal, RHO0));
    HIPCHK3(c, launch3_update_p(c->stream, c->p, c->z, c->scal, RHO0, -1, V));
    while (it < maxit) {
      if ((rc = apply3(c, c->p, c->q))) return rc;
      HIPCHK3(c, launch3_dot(c->stream, c->p, c->q, V, c->part, 3, c->scal, SIG));
      HIPCHK3(c, launch3_update_xr(c->stream, x, c->r, c->p, c->q, c->scal, RHO0 + (it & 1), SIG, V));
      HIPCHK3(c, launch3_dot(c->stream, c->r, c->r, V, c->part, 1, c->scal, RR));
      ++it;
      if ((rc = read_rr(&rr, &bb))) return rc;
      if (!std::isfinite(rr)) return fail3(c, PICS_ERR_NONFINITE, "3D PCG: non-finite residual");
      if (rr <= tol * tol * bb) {
        status = 1;
        break;
      }
      if ((rc = z_of(c->z))) return rc;
      HIPCHK3(c, launch3_dot(c->stream, c->r, c->z, V, c->part, 2, c->scal, RHO0 + (it & 1)));
      HIPCHK3(c, launch3_update_p(c->stream, c->p, c->z, c->scal, RHO0 + (it & 1), RHO0 + ((it - 1) & 1), V));
    }
  }
  if (iters_out) *iters_out = it;
  if (relres_out) *relres_out = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
  return status == 1 ? PICS_OK : (tol > 0.0 ? PICS_WARN_MAXIT : PICS_OK);
}

}  // extern "C"
