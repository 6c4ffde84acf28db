// Per-launch timing of the main kernels with HIP events recorded on the
// stream each kernel is launched on.  A solve activates the handle's timer
// for the calling thread; launchers bracket their kernel with kt_begin /
// kt_end, which do nothing while no timer is active.  A timer restricted to
// whole-phase kernels (one launch per solve) records only those, so that
// the thousands of small launches of a solve carry no event overhead.  After the stream has
// been synchronized the records are folded into per-kernel totals of time,
// algorithmic flops and algorithmic bytes.
#include <map>
#include <string>
#include <vector>

#include "hsdm_internal.h"

struct KtRec {
  int id;
  double flops, bytes;
  int nbound;  // > 0: work scales with a device-side count bounded by nbound
  hipEvent_t e0, e1;
  int tag;
};

struct KTimer {
  std::vector<std::string> names;
  std::map<std::string, int> ids;
  std::vector<KtRec> recs;
  std::vector<hipEvent_t> pool;
  std::vector<double> ms, flops, bytes;
  std::vector<long> launches;
  bool whole_only = false;  // record only launches marked whole-phase
  std::string only;         // non-empty: record only launches of this kernel
  bool pending = false;     // the last kt_begin recorded an event
};

namespace {
thread_local KTimer* kt_cur = nullptr;
thread_local int kt_tag = -1;

hipEvent_t take_event(KTimer* k) {
  if (!k->pool.empty()) {
    hipEvent_t e = k->pool.back();
    k->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

KTimer* kt_create() { return new KTimer(); }

void kt_destroy(KTimer* k) {
  if (!k) return;
  kt_reset(k);
  for (hipEvent_t e : k->pool) (void)hipEventDestroy(e);
  delete k;
}

void kt_activate(KTimer* k) { kt_cur = k; }

void kt_set_tag(int t) { kt_tag = t; }

void kt_set_last_work(const char* name, double flops, double bytes) {
  KTimer* k = kt_cur;
  if (!k) return;
  auto it = k->ids.find(name);
  if (it == k->ids.end()) return;
  for (auto r = k->recs.rbegin(); r != k->recs.rend(); ++r)
    if (r->id == it->second) {
      r->flops = flops;
      r->bytes = bytes;
      r->nbound = 0;
      return;
    }
}

void kt_set_whole_only(KTimer* k, bool on) {
  if (k) k->whole_only = on;
}

void kt_set_only(KTimer* k, const char* name) {
  if (k) k->only = name ? name : "";
}

void kt_reset(KTimer* k) {
  if (!k) return;
  for (KtRec& r : k->recs) {
    if (r.e0) k->pool.push_back(r.e0);
    if (r.e1) k->pool.push_back(r.e1);
  }
  k->recs.clear();
  std::fill(k->ms.begin(), k->ms.end(), 0.0);
  std::fill(k->flops.begin(), k->flops.end(), 0.0);
  std::fill(k->bytes.begin(), k->bytes.end(), 0.0);
  std::fill(k->launches.begin(), k->launches.end(), 0L);
}

void kt_begin(const char* name, double flops, double bytes, int nbound, hipStream_t s,
              bool whole_phase) {
  KTimer* k = kt_cur;
  if (!k) return;
  k->pending = false;
  if (k->whole_only && !whole_phase) return;
  if (!k->only.empty() && k->only != name) return;
  auto it = k->ids.find(name);
  int id;
  if (it == k->ids.end()) {
    id = (int)k->names.size();
    k->names.emplace_back(name);
    k->ids[name] = id;
    k->ms.push_back(0.0);
    k->flops.push_back(0.0);
    k->bytes.push_back(0.0);
    k->launches.push_back(0);
  } else {
    id = it->second;
  }
  KtRec r{id, flops, bytes, nbound, take_event(k), nullptr, kt_tag};
  if (r.e0) (void)hipEventRecord(r.e0, s);
  k->recs.push_back(r);
  k->pending = true;
}

void kt_end(hipStream_t s) {
  KTimer* k = kt_cur;
  if (!k || !k->pending || k->recs.empty()) return;
  k->pending = false;
  KtRec& r = k->recs.back();
  r.e1 = take_event(k);
  if (r.e1) (void)hipEventRecord(r.e1, s);
}

void kt_collect(KTimer* k, int m, const int* tag_m, int ntag) {
  if (!k) return;
  for (KtRec& r : k->recs) {
    float t = 0.f;
    if (r.e0 && r.e1 && hipEventElapsedTime(&t, r.e0, r.e1) == hipSuccess) k->ms[r.id] += t;
    const int mr = (tag_m && r.tag >= 0 && r.tag < ntag) ? tag_m[r.tag] : m;
    const double sc = (r.nbound > 0 && mr >= 0) ? (double)mr / r.nbound : 1.0;
    k->flops[r.id] += r.flops * sc;
    k->bytes[r.id] += r.bytes * sc;
    k->launches[r.id] += 1;
    if (r.e0) k->pool.push_back(r.e0);
    if (r.e1) k->pool.push_back(r.e1);
  }
  k->recs.clear();
}

int kt_count(const KTimer* k) { return k ? (int)k->names.size() : 0; }

const char* kt_stat(const KTimer* k, int i, double* out) {
  if (!k || i < 0 || i >= (int)k->names.size()) return nullptr;
  if (out) {
    out[0] = k->ms[i];
    out[1] = k->flops[i];
    out[2] = k->bytes[i];
    out[3] = (double)k->launches[i];
  }
  return k->names[i].c_str();
}
