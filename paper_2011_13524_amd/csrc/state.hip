// State handles, error reporting, uploads, initialisation and host transfer
// (section 4.2: initialization, load, copy, get_vector).
#include <cstdarg>
#include <cstdio>

#include <algorithm>

#include "dev_common.h"
#include "qsv_internal.h"

namespace qsv {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = 0; }

const char* last_error() { return g_err; }

// ------------------------------------------------------------------ Uploader

int Uploader::init() {
  if (ready_) return QSV_OK;
  if (hipHostMalloc(reinterpret_cast<void**>(&host_), kSlotBytes * kSlots, hipHostMallocDefault) !=
      hipSuccess) {
    host_ = nullptr;
    return fail(QSV_ENOMEM, "pinned upload buffer allocation failed");
  }
  if (hipMalloc(reinterpret_cast<void**>(&dev_), kSlotBytes * kSlots) != hipSuccess) {
    (void)hipHostFree(host_);
    host_ = nullptr;
    dev_ = nullptr;
    return fail(QSV_ENOMEM, "device upload buffer allocation failed");
  }
  for (int i = 0; i < kSlots; ++i) {
    if (hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming) != hipSuccess)
      return fail(QSV_EHIP, "hipEventCreate failed");
  }
  ready_ = true;
  return QSV_OK;
}

Uploader::~Uploader() {
  if (!ready_) return;
  for (int i = 0; i < kSlots; ++i) {
    if (used_[i]) (void)hipEventSynchronize(ev_[i]);
    (void)hipEventDestroy(ev_[i]);
  }
  (void)hipFree(dev_);
  (void)hipHostFree(host_);
}

int Uploader::upload(const void* src, size_t bytes, hipStream_t stream, void** dev, int* slot) {
  if (bytes > kSlotBytes) return fail(QSV_EINVAL, "upload of %zu bytes exceeds slot", bytes);
  int rc = init();
  if (rc) return rc;
  const int s = next_;
  next_ = (next_ + 1) % kSlots;
  if (used_[s]) QSV_HIP_CHECK(hipEventSynchronize(ev_[s]));
  std::memcpy(host_ + s * kSlotBytes, src, bytes);
  QSV_HIP_CHECK(hipMemcpyAsync(dev_ + s * kSlotBytes, host_ + s * kSlotBytes, bytes,
                               hipMemcpyHostToDevice, stream));
  *dev = dev_ + s * kSlotBytes;
  *slot = s;
  return QSV_OK;
}

int Uploader::release(int slot, hipStream_t stream) {
  QSV_HIP_CHECK(hipEventRecord(ev_[slot], stream));
  used_[slot] = true;
  return QSV_OK;
}

int state_work(const qsv_state* s, size_t bytes, void** out) {
  *out = nullptr;
  if (s->work_cap < bytes || !s->work) {
    // the old buffer may still be read by enqueued work
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(QSV_EHIP, "stream synchronisation failed");
    if (s->work) (void)hipFree(s->work);
    s->work = nullptr;
    s->work_cap = 0;
    const size_t cap = std::max<size_t>(bytes, 256);
    if (hipMalloc(&s->work, cap) != hipSuccess) {
      s->work = nullptr;
      return fail(QSV_ENOMEM, "work buffer of %zu bytes: allocation failed", bytes);
    }
    s->work_cap = cap;
  }
  *out = s->work;
  return QSV_OK;
}

// ------------------------------------------------------------------ kernels

// Zero the state and set amplitude k to one: the computational basis state |k>.
template <typename R>
__global__ void __launch_bounds__(256) k_set_basis(R* psi, uint64_t nvec, uint64_t k) {
  // each thread writes one 16-byte vector (2 amplitudes for complex64, 1 for complex128)
  constexpr int A = sizeof(R) == 4 ? 2 : 1;
  // grid-stride: launches stay within 2^32 work-items for any state size
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < nvec; t += stride) {
    R v[4] = {0, 0, 0, 0};
    const uint64_t x0 = t * A;
    if (k >= x0 && k < x0 + A) v[2 * (k - x0)] = R(1);
    if constexpr (A == 2)
      *reinterpret_cast<float4*>(psi + 4 * t) = make_float4(v[0], v[1], v[2], v[3]);
    else
      *reinterpret_cast<double2*>(psi + 2 * t) = make_double2(v[0], v[1]);
  }
}

int check_state(const qsv_state* s) {
  if (!s) return fail(QSV_EINVAL, "null state");
  if (!s->ptr) return fail(QSV_EINVAL, "state has no memory");
  return QSV_OK;
}

int ensure_reduce_scratch(qsv_state* s, size_t doubles) {
  if (s->red_cap >= doubles) return QSV_OK;
  if (s->red) {
    QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
    (void)hipFree(s->red);
    (void)hipHostFree(s->red_host);
    s->red = nullptr;
    s->red_host = nullptr;
    s->red_cap = 0;
  }
  if (hipMalloc(reinterpret_cast<void**>(&s->red), doubles * sizeof(double)) != hipSuccess)
    return fail(QSV_ENOMEM, "reduction scratch allocation failed");
  if (hipHostMalloc(reinterpret_cast<void**>(&s->red_host), doubles * sizeof(double),
                    hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(s->red);
    s->red = nullptr;
    return fail(QSV_ENOMEM, "pinned reduction buffer allocation failed");
  }
  s->red_cap = doubles;
  return QSV_OK;
}

static int set_basis_impl(qsv_state* s, uint64_t k) {
  const uint64_t N = dim(s->n);
  const uint64_t nvec = s->dtype == QSV_C64 ? (N + 1) / 2 : N;
  const dim3 grid(unsigned(std::min<uint64_t>((nvec + 255) / 256, uint64_t(1) << 22)));
  if (s->dtype == QSV_C64) {
    hipLaunchKernelGGL(k_set_basis<float>, grid, dim3(256), 0, s->stream,
                       static_cast<float*>(s->ptr), nvec, k);
  } else {
    hipLaunchKernelGGL(k_set_basis<double>, grid, dim3(256), 0, s->stream,
                       static_cast<double*>(s->ptr), nvec, k);
  }
  QSV_HIP_CHECK(hipGetLastError());
  return QSV_OK;
}

static int check_device() {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
    return fail(QSV_ENODEV, "no HIP device available");
  return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

const char* qsv_last_error(void) { return qsv::last_error(); }

int qsv_version(void) { return 100; }

int qsv_state_alloc(int n, qsv_dtype dtype, void* stream, qsv_state** out) {
  clear_error();
  if (!out) return fail(QSV_EINVAL, "null output handle");
  *out = nullptr;
  if (n < 1 || n > 34) return fail(QSV_ERANGE, "qubit count %d outside [1, 34]", n);
  if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_EDTYPE, "unknown dtype %d", int(dtype));
  int rc = check_device();
  if (rc) return rc;
  const size_t bytes = dim(n) * amp_bytes(dtype);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QSV_ENOMEM, "cannot allocate %zu bytes for a %d-qubit state", bytes, n);
  }
  qsv_state* s = new (std::nothrow) qsv_state();
  if (!s) {
    (void)hipFree(p);
    return fail(QSV_ENOMEM, "host allocation failed");
  }
  s->ptr = p;
  s->n = n;
  s->dtype = dtype;
  s->stream = static_cast<hipStream_t>(stream);
  s->owned = true;
  (void)hipGetDevice(&s->device);
  rc = set_basis_impl(s, 0);
  if (rc) {
    (void)hipFree(p);
    delete s;
    return rc;
  }
  *out = s;
  return QSV_OK;
}

int qsv_state_wrap(void* dev_ptr, int n, qsv_dtype dtype, void* stream, qsv_state** out) {
  clear_error();
  if (!out) return fail(QSV_EINVAL, "null output handle");
  *out = nullptr;
  if (!dev_ptr) return fail(QSV_EINVAL, "null device pointer");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 16 != 0)
    return fail(QSV_EINVAL, "device pointer must be 16-byte aligned");
  if (n < 1 || n > 34) return fail(QSV_ERANGE, "qubit count %d outside [1, 34]", n);
  if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_EDTYPE, "unknown dtype %d", int(dtype));
  qsv_state* s = new (std::nothrow) qsv_state();
  if (!s) return fail(QSV_ENOMEM, "host allocation failed");
  s->ptr = dev_ptr;
  s->n = n;
  s->dtype = dtype;
  s->stream = static_cast<hipStream_t>(stream);
  s->owned = false;
  (void)hipGetDevice(&s->device);
  *out = s;
  return QSV_OK;
}

int qsv_state_free(qsv_state* s) {
  clear_error();
  if (!s) return QSV_OK;
  (void)hipStreamSynchronize(s->stream);
  if (s->owned && s->ptr) (void)hipFree(s->ptr);
  if (s->red) (void)hipFree(s->red);
  if (s->red_host) (void)hipHostFree(s->red_host);
  if (s->big) (void)hipFree(s->big);
  if (s->work) (void)hipFree(s->work);
  delete s;
  return QSV_OK;
}

int qsv_state_info(const qsv_state* s, int* n, int* dtype, void** dev_ptr) {
  clear_error();
  if (!s) return fail(QSV_EINVAL, "null state");
  if (n) *n = s->n;
  if (dtype) *dtype = int(s->dtype);
  if (dev_ptr) *dev_ptr = s->ptr;
  return QSV_OK;
}

int qsv_state_sync(const qsv_state* s) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
  return QSV_OK;
}

int qsv_set_basis(qsv_state* s, uint64_t k) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  if (k >= dim(s->n)) return fail(QSV_ERANGE, "basis index out of range for %d qubits", s->n);
  return set_basis_impl(s, k);
}

int qsv_load(qsv_state* s, const double* host) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  if (!host) return fail(QSV_EINVAL, "null host buffer");
  const uint64_t nreal = 2 * dim(s->n);
  if (s->dtype == QSV_C128) {
    QSV_HIP_CHECK(hipMemcpyAsync(s->ptr, host, nreal * sizeof(double), hipMemcpyHostToDevice,
                                 s->stream));
    QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
    return QSV_OK;
  }
  // complex64: narrow on the host in bounded chunks
  const uint64_t chunk = uint64_t(1) << 24;
  std::vector<float> tmp(size_t(std::min(chunk, nreal)));
  for (uint64_t off = 0; off < nreal; off += chunk) {
    const uint64_t cnt = std::min(chunk, nreal - off);
    for (uint64_t i = 0; i < cnt; ++i) tmp[i] = float(host[off + i]);
    QSV_HIP_CHECK(hipMemcpyAsync(static_cast<float*>(s->ptr) + off, tmp.data(), cnt * sizeof(float),
                                 hipMemcpyHostToDevice, s->stream));
    QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
  }
  return QSV_OK;
}

int qsv_store(const qsv_state* s, double* host) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  if (!host) return fail(QSV_EINVAL, "null host buffer");
  const uint64_t nreal = 2 * dim(s->n);
  if (s->dtype == QSV_C128) {
    QSV_HIP_CHECK(hipMemcpyAsync(host, s->ptr, nreal * sizeof(double), hipMemcpyDeviceToHost,
                                 s->stream));
    QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
    return QSV_OK;
  }
  const uint64_t chunk = uint64_t(1) << 24;
  std::vector<float> tmp(size_t(std::min(chunk, nreal)));
  for (uint64_t off = 0; off < nreal; off += chunk) {
    const uint64_t cnt = std::min(chunk, nreal - off);
    QSV_HIP_CHECK(hipMemcpyAsync(tmp.data(), static_cast<const float*>(s->ptr) + off,
                                 cnt * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    QSV_HIP_CHECK(hipStreamSynchronize(s->stream));
    for (uint64_t i = 0; i < cnt; ++i) host[off + i] = double(tmp[i]);
  }
  return QSV_OK;
}

int qsv_copy(qsv_state* dst, const qsv_state* src) {
  clear_error();
  int rc = check_state(dst);
  if (rc) return rc;
  rc = check_state(src);
  if (rc) return rc;
  if (dst->n != src->n) return fail(QSV_ERANGE, "qubit counts differ (%d vs %d)", dst->n, src->n);
  if (dst->dtype != src->dtype) return fail(QSV_EDTYPE, "dtypes differ");
  if (dst->ptr == src->ptr) return QSV_OK;
  // order the copy after work already enqueued on the source's stream
  if (src->stream != dst->stream) QSV_HIP_CHECK(hipStreamSynchronize(src->stream));
  QSV_HIP_CHECK(hipMemcpyAsync(dst->ptr, src->ptr, dim(dst->n) * amp_bytes(dst->dtype),
                               hipMemcpyDeviceToDevice, dst->stream));
  return QSV_OK;
}

}  // extern "C"
