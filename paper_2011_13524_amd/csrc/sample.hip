// Sampling of Z-basis outcomes (section 4.2.2: sampling goes through a
// cumulative distribution built as pre-processing, an extra 2^n-long array).
//
// For a uniform u in [0, 1) the sample is the smallest basis index x with
// C(x) > u * C(N - 1), C the inclusive cumulative sum of |psi|^2 in FP64.
//
// The cumulative distribution is a tree of local scans. Level 0 holds, for
// every chunk of 4096 amplitudes, the inclusive scan of |psi|^2 within the
// chunk (8 bytes per amplitude); level l + 1 holds the same for the chunk
// totals of level l, up to a level of one chunk, whose last entry is the
// total. A sample descends the tree with one binary search per level.
//
// Within a chunk, thread t of 256 scans its 16 consecutive entries, and the
// thread offsets B_t are chained in order, B_{t+1} = B_t + T_t (T_t the
// thread's sum), by one thread. Every stored value is then B_t + run, and the
// first value of a thread equals the last of the previous one plus its own
// entry with the same rounding, so a stored scan is non-decreasing and rises
// only at entries of nonzero probability: a search never lands on an outcome
// of probability zero.
#include <algorithm>
#include <vector>

#include "dev_common.h"
#include "qsv_internal.h"

namespace qsv {

constexpr int kScanThreads = 256;
constexpr int kScanChunkBits = 12;
constexpr uint32_t kScanChunk = 1u << kScanChunkBits;
constexpr uint32_t kScanPer = kScanChunk / kScanThreads;  // 16
constexpr int kScanMaxLevels = 4;                          // 4 x 12 bits >= 34 qubits
constexpr int kSampleThreads = 256;

struct ScanTree {
  const double* cdf[kScanMaxLevels];
  uint64_t count[kScanMaxLevels];
  int levels;
};

template <typename R>
__device__ __forceinline__ double scan_weight(const R* psi, uint64_t i) {
  const cx<R> v = load1(psi, i);
  const double re = v.re, im = v.im;
  return re * re + im * im;
}

// AMP: `in` holds amplitudes of type R (weights |psi|^2); otherwise `in` holds
// doubles (R == double) taken as they are. One workgroup per chunk of
// kScanChunk entries (the last chunk may be short); cdf receives the chunk's
// local inclusive scan and sums[blockIdx.x] its total (the last scan value).
// cdf may alias in: the chunk is read whole before it is written.
//
// The chunk passes through LDS so that global reads and writes stay
// coalesced; entry j sits at j + j / 16 (one pad slot per thread's run of 16)
// so that the per-thread runs fall in different banks.
__device__ __forceinline__ uint32_t scan_slot(uint32_t j) { return j + (j >> 4); }

template <typename R, bool AMP>
__global__ void __launch_bounds__(kScanThreads)
    k_scan_chunks(const R* in, uint64_t count, double* cdf, double* __restrict__ sums) {
  __shared__ double p[kScanChunk + kScanChunk / kScanPer];
  __shared__ double base[kScanThreads];
  const uint64_t first = uint64_t(blockIdx.x) << kScanChunkBits;
  const uint32_t len = uint32_t(min<uint64_t>(kScanChunk, count - first));
  const uint32_t tid = threadIdx.x;
  // a full chunk of amplitudes moves as 16-byte vectors, two entries per lane
  const bool full = AMP && len == kScanChunk;
  if (full) {
    if constexpr (AMP) {
#pragma unroll
      for (uint32_t i = 0; i < kScanChunk / (2 * kScanThreads); ++i) {
        const uint32_t j = 2 * (tid + i * kScanThreads);
        cx<R> v[2];
        AmpIO<R, 2>::load(in, first + j, v);
        p[scan_slot(j)] = double(v[0].re) * double(v[0].re) + double(v[0].im) * double(v[0].im);
        p[scan_slot(j + 1)] = double(v[1].re) * double(v[1].re) + double(v[1].im) * double(v[1].im);
      }
    }
  } else {
    for (uint32_t j = tid; j < len; j += kScanThreads) {
      if constexpr (AMP)
        p[scan_slot(j)] = scan_weight(in, first + j);
      else
        p[scan_slot(j)] = double(in[first + j]);
    }
  }
  __syncthreads();
  // thread t's entries 16t .. 16t + 15, scanned in registers
  const uint32_t j0 = tid * kScanPer;
  double run[kScanPer];
  double acc = 0.0;
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; ++k) {
    if (j0 + k < len) acc += p[scan_slot(j0 + k)];
    run[k] = acc;
  }
  base[tid] = acc;  // thread total T_t (0 past the end)
  __syncthreads();
  // B_0 = 0, B_{t+1} = B_t + T_t, in order; 16 loads in flight per step
  if (tid == 0) {
    double b = 0.0;
    for (uint32_t t0 = 0; t0 < kScanThreads; t0 += 16) {
      double T[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) T[k] = base[t0 + k];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        base[t0 + k] = b;
        b += T[k];
      }
    }
  }
  __syncthreads();
  const double b = base[tid];
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; ++k)
    if (j0 + k < len) p[scan_slot(j0 + k)] = b + run[k];
  __syncthreads();
  if (full) {
#pragma unroll
    for (uint32_t i = 0; i < kScanChunk / (2 * kScanThreads); ++i) {
      const uint32_t j = 2 * (tid + i * kScanThreads);  // j and j + 1 share a run: adjacent slots
      nt_store(f64x2{p[scan_slot(j)], p[scan_slot(j + 1)]}, reinterpret_cast<f64x2*>(cdf + first + j));
    }
  } else {
    for (uint32_t j = tid; j < len; j += kScanThreads) cdf[first + j] = p[scan_slot(j)];
  }
  if (tid == 0) sums[blockIdx.x] = p[scan_slot(len - 1)];
}

// Smallest j in [lo, hi) with c[j] > r, given c[hi - 1] > r and c non-decreasing.
__device__ __forceinline__ uint64_t first_above(const double* c, uint64_t lo, uint64_t hi, double r) {
  uint64_t a = lo, b = hi - 1;
  while (a < b) {
    const uint64_t m = (a + b) >> 1;
    if (c[m] > r)
      b = m;
    else
      a = m + 1;
  }
  return a;
}

__global__ void __launch_bounds__(kSampleThreads)
    k_sample(ScanTree T, const double* __restrict__ u, uint64_t count, int64_t* __restrict__ out) {
  const uint64_t i = uint64_t(blockIdx.x) * kSampleThreads + threadIdx.x;
  if (i >= count) return;
  const int top = T.levels - 1;
  double r = u[i] * T.cdf[top][T.count[top] - 1];
  uint64_t seg = 0;
  for (int l = top; l >= 0; --l) {
    const double* c = T.cdf[l];
    const uint64_t lo = seg << kScanChunkBits;
    const uint64_t hi = min<uint64_t>(lo + kScanChunk, T.count[l]);
    const double tot = c[hi - 1];  // > 0: the segment was reached through a rise
    if (!(r < tot)) r = nextafter(tot, 0.0);
    const uint64_t a = first_above(c, lo, hi, r);
    if (a > lo) r -= c[a - 1];  // >= 0: c[a - 1] <= r
    seg = a;
  }
  out[i] = int64_t(seg);
}

namespace {

// Device memory of one sampling call, carved from the state's work buffer
// (kept for the next call; every call synchronises before returning).
struct SampleBuffers {
  char* base = nullptr;
  size_t used = 0, cap = 0;
  template <typename T>
  T* get(size_t n) {
    const size_t bytes = (std::max<size_t>(n, 1) * sizeof(T) + 255) / 256 * 256;
    if (used + bytes > cap) return nullptr;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

template <typename R>
int sample_t(const qsv_state* s, const double* u, int64_t count, int64_t* out) {
  hipStream_t st = s->stream;
  // sizes: level 0 table (one FP64 per amplitude), the chunk totals of every
  // level, then the uniforms and the outputs
  size_t need = 0;
  auto add = [&need](size_t bytes) { need += (std::max<size_t>(bytes, 1) + 255) / 256 * 256; };
  {
    uint64_t c = dim(s->n);
    add(c * sizeof(double));
    do {
      c = (c + kScanChunk - 1) >> kScanChunkBits;
      add(c * sizeof(double));
    } while (c > 1);
    add(size_t(count) * sizeof(double));
    add(size_t(count) * sizeof(int64_t));
  }
  SampleBuffers buf;
  void* wb = nullptr;
  if (int rc = state_work(s, need, &wb)) return rc;
  buf.base = static_cast<char*>(wb);
  buf.cap = need;
  ScanTree T{};
  uint64_t cnt = dim(s->n);
  // level 0: |psi|^2 chunks of the state; higher levels scan the chunk totals in place
  double* level_cdf = buf.get<double>(cnt);
  if (!level_cdf) return fail(QSV_ENOMEM, "cumulative table allocation failed");
  uint64_t chunks = (cnt + kScanChunk - 1) >> kScanChunkBits;
  double* sums = buf.get<double>(chunks);
  if (!sums) return fail(QSV_ENOMEM, "cumulative table allocation failed");
  hipLaunchKernelGGL((k_scan_chunks<R, true>), dim3(unsigned(chunks)), dim3(kScanThreads), 0, st,
                     static_cast<const R*>(s->ptr), cnt, level_cdf, sums);
  QSV_HIP_CHECK(hipGetLastError());
  T.cdf[0] = level_cdf;
  T.count[0] = cnt;
  T.levels = 1;
  while (chunks > 1) {
    if (T.levels == kScanMaxLevels) return fail(QSV_ERANGE, "state too large for the sampling table");
    cnt = chunks;
    double* in = sums;
    chunks = (cnt + kScanChunk - 1) >> kScanChunkBits;
    sums = buf.get<double>(chunks);
    if (!sums) return fail(QSV_ENOMEM, "cumulative table allocation failed");
    hipLaunchKernelGGL((k_scan_chunks<double, false>), dim3(unsigned(chunks)), dim3(kScanThreads), 0,
                       st, in, cnt, in, sums);
    QSV_HIP_CHECK(hipGetLastError());
    T.cdf[T.levels] = in;
    T.count[T.levels] = cnt;
    ++T.levels;
  }
  double total = 0.0;
  QSV_HIP_CHECK(hipMemcpyAsync(&total, sums, sizeof(double), hipMemcpyDeviceToHost, st));
  QSV_HIP_CHECK(hipStreamSynchronize(st));
  if (!(total > 0.0)) return fail(QSV_EINVAL, "state has zero norm");
  if (count == 0) return QSV_OK;
  double* du = buf.get<double>(size_t(count));
  int64_t* dout = buf.get<int64_t>(size_t(count));
  if (!du || !dout) return fail(QSV_ENOMEM, "sample buffer allocation failed");
  QSV_HIP_CHECK(hipMemcpyAsync(du, u, size_t(count) * sizeof(double), hipMemcpyHostToDevice, st));
  const uint64_t blocks = (uint64_t(count) + kSampleThreads - 1) / kSampleThreads;
  hipLaunchKernelGGL(k_sample, dim3(unsigned(blocks)), dim3(kSampleThreads), 0, st, T, du,
                     uint64_t(count), dout);
  QSV_HIP_CHECK(hipGetLastError());
  QSV_HIP_CHECK(hipMemcpyAsync(out, dout, size_t(count) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  QSV_HIP_CHECK(hipStreamSynchronize(st));
  return QSV_OK;
}

}  // namespace

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_sample(const qsv_state* s, const double* u, int64_t count, int64_t* out) {
  clear_error();
  int rc = check_state(s);
  if (rc) return rc;
  if (count < 0) return fail(QSV_EINVAL, "negative sample count");
  if (count > (int64_t(1) << 31)) return fail(QSV_ERANGE, "at most 2^31 samples per call");
  if (count > 0 && (!u || !out)) return fail(QSV_EINVAL, "null argument");
  for (int64_t i = 0; i < count; ++i)
    if (!(u[i] >= 0.0 && u[i] < 1.0)) return fail(QSV_ERANGE, "uniform %lld outside [0, 1)", (long long)i);
  return s->dtype == QSV_C64 ? sample_t<float>(s, u, count, out) : sample_t<double>(s, u, count, out);
}

}  // extern "C"
