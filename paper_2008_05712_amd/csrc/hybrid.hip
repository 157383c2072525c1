// Dynamic CPU/GPU scheduling of work requests (Sec. 3.3) and the CPU kernel it needs for the
// Lennard-Jones cell-pair requests.  Host code only.
//
// The policy: a request's workload is the number of input data items it reads (for a cell pair:
// the records of both cells).  After each execution on either device the caller records the
// items and the time; each device keeps the running mean of its seconds per item over its
// executions.  A queue of requests is split so that the CPU gets a share
// tau_gpu / (tau_cpu + tau_gpu) of the items (equal finishing times): the requests are scanned
// from the front with a running sum of their items, and the prefix up to the request at which the
// sum reaches the CPU's share goes to the CPU, the rest to the GPU.  Until both devices have been
// timed the share is one half, so the first requests run on both.
#include <algorithm>
#include <cmath>
#include <new>
#include <thread>
#include <vector>

#include "gc_internal.h"

struct gc_hybrid_ {
  double tau[2] = {0.0, 0.0};  // running mean seconds per item: CPU, GPU
  int64_t runs[2] = {0, 0};
};

extern "C" gc_status gc_hybrid_create(gc_hybrid* out) {
  if (!out) return GC_E_INVAL;
  gc_hybrid h = new (std::nothrow) gc_hybrid_();
  if (!h) return GC_E_NOMEM;
  *out = h;
  return GC_OK;
}

extern "C" gc_status gc_hybrid_destroy(gc_hybrid h) {
  if (!h) return GC_E_INVAL;
  delete h;
  return GC_OK;
}

extern "C" gc_status gc_hybrid_record(gc_hybrid h, int32_t device, int64_t items, double seconds) {
  if (!h || (device != GC_DEVICE_CPU && device != GC_DEVICE_GPU) || items < 1 || !(seconds >= 0.0))
    return GC_E_INVAL;
  const double x = seconds / (double)items;
  const int64_t k = ++h->runs[device];
  h->tau[device] += (x - h->tau[device]) / (double)k;
  return GC_OK;
}

extern "C" gc_status gc_hybrid_split(gc_hybrid h, const int64_t* items, int32_t n, int32_t* n_cpu,
                                     int64_t* items_cpu) {
  if (!h || n < 0 || (n > 0 && !items) || !n_cpu) return GC_E_INVAL;
  double total = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    if (items[i] < 0) return GC_E_INVAL;
    total += (double)items[i];
  }
  double share = 0.5;
  if (h->runs[GC_DEVICE_CPU] > 0 && h->runs[GC_DEVICE_GPU] > 0) {
    const double s = h->tau[GC_DEVICE_CPU] + h->tau[GC_DEVICE_GPU];
    share = s > 0.0 ? h->tau[GC_DEVICE_GPU] / s : 0.5;
  }
  const double want = total * share;
  int32_t k = 0;
  int64_t cum = 0;
  if (want > 0.0) {
    k = n;
    for (int32_t i = 0; i < n; ++i) {
      cum += items[i];
      if ((double)cum >= want) {
        k = i + 1;
        break;
      }
    }
  }
  int64_t ic = 0;
  for (int32_t i = 0; i < k; ++i) ic += items[i];
  *n_cpu = k;
  if (items_cpu) *items_cpu = ic;
  return GC_OK;
}

extern "C" gc_status gc_hybrid_state(gc_hybrid h, double* tau_cpu, double* tau_gpu, int64_t* runs_cpu,
                                     int64_t* runs_gpu) {
  if (!h) return GC_E_INVAL;
  if (tau_cpu) *tau_cpu = h->tau[GC_DEVICE_CPU];
  if (tau_gpu) *tau_gpu = h->tau[GC_DEVICE_GPU];
  if (runs_cpu) *runs_cpu = h->runs[GC_DEVICE_CPU];
  if (runs_gpu) *runs_gpu = h->runs[GC_DEVICE_GPU];
  return GC_OK;
}

// ---------------------------------------------------------------- CPU Lennard-Jones kernel

namespace {

// One cell-pair task on the CPU: the device's FP32 cutoff decision and force factor, both atoms
// updated, sums in FP64 per thread.
void lj_task_cpu(const gc_task& tk, int32_t jb, int32_t jn, const float* rec, int32_t nt, const float* e24,
                 const float* sg2, float rc2, double* F) {
  const float ax = tk.shift[0] > 0.f ? tk.shift[0] : 0.f, ay = tk.shift[1] > 0.f ? tk.shift[1] : 0.f,
              az = tk.shift[2] > 0.f ? tk.shift[2] : 0.f;
  const float bx = tk.shift[0] < 0.f ? tk.shift[0] : 0.f, by = tk.shift[1] < 0.f ? tk.shift[1] : 0.f,
              bz = tk.shift[2] < 0.f ? tk.shift[2] : 0.f;
  const bool self = (tk.flags & GC_TASK_SELF) != 0;
  for (int32_t i = tk.i_begin; i < tk.i_begin + tk.i_count; ++i) {
    const float* xi = rec + 4 * (size_t)i;
    const float pxi = xi[0] - ax, pyi = xi[1] - ay, pzi = xi[2] - az;
    const int ti = (int)xi[3];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int32_t j = self ? i + 1 : jb; j < jb + jn; ++j) {
      const float* xj = rec + 4 * (size_t)j;
      const float dx = pxi - (xj[0] + bx), dy = pyi - (xj[1] + by), dz = pzi - (xj[2] + bz);
      const float r2 = std::fma(dz, dz, std::fma(dy, dy, dx * dx));
      if (!(r2 < rc2)) continue;
      const int k = ti * nt + (int)xj[3];
      const float ri2 = 1.f / r2;
      const float q = sg2[k] * ri2;
      const float q3 = q * q * q;
      const float f = e24[k] * q3 * (2.f * q3 - 1.f) * ri2;
      fx += (double)(f * dx);
      fy += (double)(f * dy);
      fz += (double)(f * dz);
      double* Fj = F + 3 * (size_t)j;
      Fj[0] -= (double)(f * dx);
      Fj[1] -= (double)(f * dy);
      Fj[2] -= (double)(f * dz);
    }
    double* Fi = F + 3 * (size_t)i;
    Fi[0] += fx;
    Fi[1] += fy;
    Fi[2] += fz;
  }
}

}  // namespace

extern "C" gc_status gc_lj_forces_cpu(const gc_task* tasks, int32_t n_tasks, const int32_t* j_ranges, int32_t n_ranges,
                                      const float* rec, int32_t n_ids, int32_t n_types, const float* eps_t,
                                      const float* sig_t, const float* mass_t, float r_cut, float* acc,
                                      int32_t n_threads) {
  if (n_tasks < 0 || n_ids < 0 || (n_tasks > 0 && (!tasks || !j_ranges || !rec || !acc)) || n_types < 1 ||
      n_types > 8 || !eps_t || !sig_t || !mass_t || !(r_cut > 0.f) || n_threads < 0)
    return GC_E_INVAL;
  for (int32_t t = 0; t < n_tasks; ++t) {
    const gc_task& tk = tasks[t];
    if (tk.j_nranges != 1 || tk.j_first < 0 || tk.j_first >= n_ranges || tk.i_begin < 0 || tk.i_count < 0 ||
        (int64_t)tk.i_begin + tk.i_count > n_ids)
      return GC_E_INVAL;
    const int32_t jb = j_ranges[2 * tk.j_first], jn = j_ranges[2 * tk.j_first + 1];
    if (jb < 0 || jn < 0 || (int64_t)jb + jn > n_ids) return GC_E_INVAL;
    if ((tk.flags & GC_TASK_SELF) && (jb != tk.i_begin || jn != tk.i_count)) return GC_E_INVAL;
  }
  for (int32_t i = 0; i < n_ids; ++i) {
    const int ty = (int)rec[4 * (size_t)i + 3];
    if (ty < 0 || ty >= n_types) return GC_E_INVAL;
  }
  float e24[64], sg2[64];
  for (int a = 0; a < n_types; ++a)
    for (int b = 0; b < n_types; ++b) {
      const float s = 0.5f * (sig_t[a] + sig_t[b]);
      e24[a * n_types + b] = 24.f * std::sqrt(eps_t[a] * eps_t[b]);
      sg2[a * n_types + b] = s * s;
    }
  const float rc2 = r_cut * r_cut;
  int nth = n_threads > 0 ? n_threads : (int)std::thread::hardware_concurrency();
  nth = std::max(1, std::min(nth, 64));
  // every thread sums into its own array over all ids (reduced at the end): at least 256 tasks each
  nth = std::max(1, std::min<int>(nth, n_tasks / 256));
  std::vector<std::vector<double>> part;
  try {
    part.assign(nth, std::vector<double>(3 * (size_t)n_ids, 0.0));
  } catch (const std::bad_alloc&) {
    return GC_E_NOMEM;
  }
  auto work = [&](int w) {
    const int32_t t0 = (int32_t)((int64_t)n_tasks * w / nth), t1 = (int32_t)((int64_t)n_tasks * (w + 1) / nth);
    for (int32_t t = t0; t < t1; ++t) {
      const gc_task& tk = tasks[t];
      lj_task_cpu(tk, j_ranges[2 * tk.j_first], j_ranges[2 * tk.j_first + 1], rec, n_types, e24, sg2, rc2,
                  part[w].data());
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < nth; ++w) pool.emplace_back(work, w);
  work(0);
  for (auto& th : pool) th.join();
  // threads' sums in a fixed order; a = F / m
  for (int32_t i = 0; i < n_ids; ++i) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int w = 0; w < nth; ++w)
      for (int d = 0; d < 3; ++d) s[d] += part[w][3 * (size_t)i + d];
    const double m = mass_t[(int)rec[4 * (size_t)i + 3]];
    for (int d = 0; d < 3; ++d) acc[4 * (size_t)i + d] += (float)(s[d] / m);
  }
  return GC_OK;
}
