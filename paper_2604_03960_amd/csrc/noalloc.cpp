// Allocation-free form of the stand-alone H_eff application (Eq. 18) for callers that cannot allocate
// device memory: code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
// Its intermediates (the S1 and S2 products, the two-site mixing matrix and, for FP32, the converted
// environments) live in one fixed device array of TNA_NOALLOC_SCRATCH_BYTES that every GPU the library
// runs on holds until the process ends.  The array's device address is taken once per device, at
// context creation, with hipGetSymbolAddress; host code uses only that address.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

using namespace tna;

namespace {

constexpr size_t kScratchBytes = TNA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

void *scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace tna {

tna_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("noalloc: device index out of range");
    return TNA_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return TNA_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    set_error(std::string("noalloc: hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
    return TNA_ERR_DEVICE;
  }
  g_scratch[device] = ptr;
  return TNA_OK;
}

}  // namespace tna

extern "C" {

tna_status tna_heff_apply_noalloc_bytes(int chi_l, int chi_r, int d, int D, int prec, size_t *bytes) {
  if (!bytes || chi_l < 1 || chi_r < 1 || d < 1 || D < 1) {
    set_error("heff_apply_noalloc_bytes: bad argument");
    return TNA_ERR_ARG;
  }
  const size_t nx = (size_t)D * d * d * chi_l * chi_r;
  const size_t el = prec == TNA_HEFF_F64 ? sizeof(double) : sizeof(float);
  size_t b = 2 * up256(el * nx) + up256(sizeof(double) * (size_t)(D * d * d) * (D * d * d));
  if (prec != TNA_HEFF_F64)
    b += up256(sizeof(float) * (size_t)chi_l * D * chi_l) + up256(sizeof(float) * (size_t)chi_r * D * chi_r);
  *bytes = b;
  return TNA_OK;
}

tna_status tna_heff_apply_noalloc(tna_ctx c, int chi_l, int chi_r, int d, int D, const double *L, const double *W1,
                                  const double *W2, const double *R, const double *theta, double *out, int prec) {
  TNA_TRY(heff_check_args(c, chi_l, chi_r, d, D, L, W1, W2, R, theta, out, prec));
  size_t need = 0;
  TNA_TRY(tna_heff_apply_noalloc_bytes(chi_l, chi_r, d, D, prec, &need));
  if (need > kScratchBytes) {
    set_error("heff_apply_noalloc: this shape needs " + std::to_string(need) + " bytes of scratch, the fixed array holds " +
              std::to_string(kScratchBytes) + " (use tna_heff_apply)");
    return TNA_ERR_ARG;
  }
  unsigned char *base = static_cast<unsigned char *>(scratch_of(c->device));
  if (!base) {
    set_error("heff_apply_noalloc: no scratch address for this device (context not created on it)");
    return TNA_ERR_DEVICE;
  }
  const size_t nx = (size_t)D * d * d * chi_l * chi_r;
  const size_t el = prec == TNA_HEFF_F64 ? sizeof(double) : sizeof(float);
  size_t off = 0;
  void *X = base + off;
  off += up256(el * nx);
  void *Z = base + off;
  off += up256(el * nx);
  double *M12 = reinterpret_cast<double *>(base + off);
  off += up256(sizeof(double) * (size_t)(D * d * d) * (D * d * d));
  hipStream_t s = c->stream;
  TNA_TRY(build_mix_matrix(0, d, D, W1, W2, M12, s));
  HeffOp op{chi_l, chi_r, d, D, L, R, M12, X, Z, prec};
  if (prec != TNA_HEFF_F64) {
    const int64_t nl = (int64_t)chi_l * D * chi_l, nr = (int64_t)chi_r * D * chi_r;
    float *Lf = reinterpret_cast<float *>(base + off);
    off += up256(sizeof(float) * (size_t)nl);
    float *Rf = reinterpret_cast<float *>(base + off);
    TNA_TRY(convert_f64_f32(L, Lf, nl, s));
    TNA_TRY(convert_f64_f32(R, Rf, nr, s));
    op.L = Lf;
    op.R = Rf;
  }
  return heff_device(op, theta, out, s);
}

}  // extern "C"
