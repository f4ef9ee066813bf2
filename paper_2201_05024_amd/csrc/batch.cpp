// Batches of detectors with different shapes: host planning of the job
// tables, the device workspace image, the launch forms of batched detection
// and their tuning.
//
// Planning: every item becomes one training job (one workgroup, its kernel
// specialisation picked by train_rows_variant, else train_variant), ordered
// by estimated cost so the longest trainings start first.  Jobs of the rows
// form get their kernel rows (one step per row) in the workspace, written by
// one data-parallel launch before the training launch.  Every item becomes a
// packing job and, if it has vectors to detect, a detection job of one of the
// two detection kernels: split-FP16 with VALU coefficients (2M <= 64, K <= 8)
// or two-contraction (wider shapes).  Each kernel gets one launch over the
// work items of its jobs (64-vector tiles, resp. 256-vector items), ordered
// by the cost of an item (dictionary size times per-entry work), most
// expensive first.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "apsm_internal.h"

struct apsm_batch {
  std::vector<apsm_batch_item_t> items;
  apsm::TrainCommon cm{};
  std::vector<apsm::TrainJob> tjobs;
  size_t train_lds = 0;
  std::vector<apsm::TrainJob> rjobs;          // rows form; glag/kw set at bind
  std::vector<size_t> rows_off;               // float offset of each rows job's glag (kw follows)
  std::vector<int4> ritems;                   // (rows job, first step, first lag) per kernel-row tile
  size_t rows_lds = 0, rows_floats = 0;
  int rows_max_m2 = 0;
  std::vector<apsm::PackJob> pjobs;
  int pack_max_cap = 0;
  std::vector<apsm::PackJob> pwjobs;           // two-contraction packing
  int pack_wide_threads = 0;
  std::vector<apsm::DetJob> djobs;
  std::vector<int2> ditems;
  std::vector<apsm::DetJob> wjobs;             // two-contraction detection
  std::vector<int2> witems;                    // grouped by padded width (one launch each)
  int wbegin[4] = {0, 0, 0, 0};                // items of width class c: [wbegin[c], wbegin[c + 1])
  std::vector<int> train_plain;      // items trained with their own launch
  size_t off_t = 0, off_rj = 0, off_ri = 0, off_p = 0, off_pw = 0, off_d = 0, off_i = 0, off_wd = 0, off_wi = 0,
         off_c = 0, off_rows = 0, bytes = 0;
  unsigned char* ws = nullptr;       // bound workspace (device)
  bool persistent = true;
  int cus = 0;                       // CUs the persistent grids occupy (0: all)
  int grid = 0;                      // CUs of the device
  uint64_t signature = 0;
};

namespace {

using namespace apsm;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int check_item(const apsm_batch_item_t& it, int window) {
  if (int rc = check_model(&it.model)) return rc;
  if (it.model.dict_cap < window) return APSM_ERR_INVALID_ARG;
  if (it.P < 1) return APSM_ERR_SHAPE;
  if ((long long)it.P * 2 > (long long)INT32_MAX / 2) return APSM_ERR_UNSUPPORTED;
  if (!it.rx_pilot || !it.sym_pilot) return APSM_ERR_INVALID_ARG;
  return check_detect_args(it.model.M2, it.model.K, it.sigma2, it.S, it.rx, it.soft, it.hard, it.modulation,
                           it.truth, it.err_count);
}

// Byte ranges [lo, hi) of device buffers.
struct Range {
  uintptr_t lo, hi;
};

void add_range(std::vector<Range>& v, const void* p, size_t bytes) {
  if (p && bytes) v.push_back({reinterpret_cast<uintptr_t>(p), reinterpret_cast<uintptr_t>(p) + bytes});
}

// True when no two buffers the batch writes overlap and no buffer it reads
// overlaps one it writes (the kernels of one launch would race on them).
bool buffers_disjoint(const std::vector<apsm_batch_item_t>& items) {
  std::vector<Range> wr, rd;
  for (const auto& it : items) {
    const apsm_model_t& m = it.model;
    const size_t S = it.S > 0 ? (size_t)it.S : 0, K = m.K, cap = m.dict_cap;
    add_range(wr, m.dict, (size_t)m.M2 * cap * 4);
    add_range(wr, m.alpha, cap * K * 4);
    add_range(wr, m.w, K * m.M2 * 4);
    add_range(wr, m.state, 4 * 4);
    add_range(wr, m.packed, packed_model_bytes(m.M2, m.K, m.dict_cap));
    add_range(wr, it.soft, S * K * 2 * 4);
    add_range(wr, it.hard, S * K);
    if (S > 0) add_range(wr, it.err_count, K * 8);
    add_range(rd, it.rx_pilot, (size_t)it.P * m.M2 * 4);
    add_range(rd, it.sym_pilot, (size_t)it.P * K * 2 * 4);
    add_range(rd, it.rx, S * m.M2 * 4);
    add_range(rd, it.truth, S * K);
  }
  std::sort(wr.begin(), wr.end(), [](const Range& a, const Range& c) { return a.lo < c.lo; });
  for (size_t i = 1; i < wr.size(); ++i)
    if (wr[i].lo < wr[i - 1].hi) return false;
  for (const Range& r : rd) {
    // the written range starting last at or before r.hi - 1 is the only one
    // (of these disjoint ranges) that can reach into r from below or inside
    auto it = std::upper_bound(wr.begin(), wr.end(), r.hi - 1, [](uintptr_t x, const Range& w) { return x < w.lo; });
    if (it != wr.begin() && std::prev(it)->hi > r.lo) return false;
  }
  return true;
}

uint64_t fnv(uint64_t h, int64_t v) {
  for (int b = 0; b < 8; ++b) {
    h ^= (uint64_t)((v >> (8 * b)) & 0xff);
    h *= 1099511628211ull;
  }
  return h;
}

// Shape mix of a batch: the tuned launch form is reused for equal mixes.
uint64_t signature_of(const std::vector<apsm_batch_item_t>& items) {
  uint64_t h = 1469598103934665603ull;
  for (const auto& it : items) {
    h = fnv(h, it.model.M2);
    h = fnv(h, it.model.K);
    h = fnv(h, it.model.dict_cap);
    h = fnv(h, it.P);
    h = fnv(h, it.S);
  }
  return h;
}

// Detection jobs and work items of the two kernels, from the kernel choice
// of each item's shape class (tuned, else the default); each list ordered
// by the cost of one work item (dictionary stages times per-entry work),
// most expensive first.
void assign_detection(apsm_batch& b) {
  const int n = (int)b.items.size();
  b.djobs.clear();
  b.ditems.clear();
  b.wjobs.clear();
  b.witems.clear();
  std::vector<int> det, wdet;
  for (int i = 0; i < n; ++i) {
    const auto& it = b.items[i];
    if (it.S <= 0) continue;
    (detect_kernel_for(it.model.M2, it.model.K) == kDetectF16 ? det : wdet).push_back(i);
  }
  std::vector<double> dcost(n, 0.0);
  for (int i : det) {
    const auto& it = b.items[i];
    const double D = std::min<double>(2.0 * it.P, it.model.dict_cap);
    dcost[i] = (std::ceil(D / 64.0) + 0.25) * (it.model.K + 6 + it.model.M2 / 16.0);
  }
  for (int i : wdet) {
    const auto& it = b.items[i];
    const double D = std::min<double>(2.0 * it.P, it.model.dict_cap);
    dcost[i] = (std::ceil(D / 64.0) + 0.25) * (6.0 * it.model.M2 / 32.0 + 1.0);
  }
  auto by_cost = [&](int a, int c) { return dcost[a] > dcost[c]; };
  std::stable_sort(det.begin(), det.end(), by_cost);
  // two-contraction jobs grouped by padded width (one launch per width), by cost within
  auto wvar = [&](int i) { return wide_detect_variant(b.items[i].model.M2); };
  std::stable_sort(wdet.begin(), wdet.end(), [&](int a, int c) {
    return wvar(a) != wvar(c) ? wvar(a) < wvar(c) : dcost[a] > dcost[c];
  });
  auto det_job = [&](const apsm_batch_item_t& it, int variant, size_t packed_off) {
    DetJob d{};
    d.packed = static_cast<const unsigned char*>(it.model.packed) + packed_off;
    d.w = it.model.w;
    d.state = it.model.state;
    d.flags = it.model.state + 3;
    d.rx = it.rx;
    d.soft = it.soft;
    d.hard = it.hard;
    d.truth = it.truth;
    d.err = reinterpret_cast<unsigned long long*>(it.err_count);
    d.cap = it.model.dict_cap;
    d.M2 = it.model.M2;
    d.K = it.model.K;
    d.S = it.S;
    d.modulation = it.modulation;
    d.c2 = kLog2e / (2.0f * it.sigma2);
    d.variant = variant;
    return d;
  };
  for (int i : det) {
    const auto& it = b.items[i];
    const int job = (int)b.djobs.size();
    b.djobs.push_back(det_job(it, detect_batch_variant(it.model.M2, it.model.K), 0));
    const int tiles = detect_tiles(it.S);
    for (int t = 0; t < tiles; ++t) b.ditems.push_back(make_int2(job, t));
  }
  for (int c = 0; c < 4; ++c) b.wbegin[c] = 0;
  for (int i : wdet) {
    const auto& it = b.items[i];
    const int job = (int)b.wjobs.size();
    b.wjobs.push_back(det_job(it, wvar(i), wide_offset(it.model.M2, it.model.K, it.model.dict_cap)));
    const int nit = wide_detect_items(it.S);
    for (int t = 0; t < nit; ++t) b.witems.push_back(make_int2(job, t));
    for (int c = wvar(i) + 1; c < 4; ++c) b.wbegin[c] = (int)b.witems.size();
  }
}

void plan(apsm_batch& b, const apsm_params_t* p) {
  const int n = (int)b.items.size();
  fill_common(p, b.cm);

  // training: longest first (steps x entries swept per step x width)
  std::vector<double> tcost(n);
  for (int i = 0; i < n; ++i) {
    const auto& it = b.items[i];
    const double T = 2.0 * it.P;
    const double D = std::min<double>(T, it.model.dict_cap);
    tcost[i] = T * (D * (it.model.M2 + it.model.K) + 64.0 * p->window);
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return tcost[a] > tcost[c]; });
  for (int i : order) {
    const auto& it = b.items[i];
    // users per rows job: all of them, or groups of four when the capacity
    // needs 16 coefficient slots per thread
    const int ku = std::min(it.model.K, train_rows_max_users(it.model.dict_cap));
    const int rv = train_rows_variant(it.model.M2, ku, it.model.dict_cap);
    if (rv < 0 && !train_in_table(it.model.M2)) {
      b.train_plain.push_back(i);
      continue;
    }
    TrainJob j{};
    j.rx = it.rx_pilot;
    j.sym = it.sym_pilot;
    j.dict = it.model.dict;
    j.alpha = it.model.alpha;
    j.w = it.model.w;
    j.state = it.model.state;
    j.P = it.P;
    j.M2 = it.model.M2;
    j.K = it.model.K;
    j.Kt = it.model.K;
    j.k0 = 0;
    j.cap = it.model.dict_cap;
    j.c2 = kLog2e / (2.0f * it.sigma2);
    if (rv >= 0) {
      // one job per group of ku users, all reading the detector's kernel rows;
      // the rows tiles name the first group's job
      const int q = (int)b.rjobs.size(), T = 2 * it.P;
      for (int k0 = 0; k0 < it.model.K; k0 += ku) {
        TrainJob g = j;
        g.k0 = k0;
        g.K = std::min(ku, it.model.K - k0);
        g.variant = train_rows_variant(g.M2, g.K, g.cap);
        b.rjobs.push_back(g);
        b.rows_off.push_back(b.rows_floats);
        b.rows_lds = std::max(b.rows_lds, train_rows_lds_bytes(p->window, g.M2, g.K));
      }
      b.rows_floats += (size_t)T * (j.cap + p->window);
      b.rows_max_m2 = std::max(b.rows_max_m2, j.M2);
      for (int n0 = 0; n0 < T; n0 += kernel_rows_tile_steps())
        for (int l0 = 0; l0 < j.cap; l0 += kernel_rows_tile_lags()) b.ritems.push_back(make_int4(q, n0, l0, 0));
      continue;
    }
    j.variant = train_variant(j.M2, j.K, p->window, j.cap);
    b.tjobs.push_back(j);
    b.train_lds = std::max(b.train_lds, train_lds_bytes(p->window, j.M2, j.K, j.cap));
  }

  // packing: dual shapes get both packed images
  for (int i = 0; i < n; ++i) {
    const auto& it = b.items[i];
    PackJob pj{};
    pj.dict = it.model.dict;
    pj.alpha = it.model.alpha;
    pj.w = it.model.w;
    pj.state = it.model.state;
    pj.packed = static_cast<unsigned char*>(it.model.packed);
    pj.cap = it.model.dict_cap;
    pj.M2 = it.model.M2;
    pj.K = it.model.K;
    if (detect_dual(pj.M2, pj.K)) {
      pj.variant = detect_batch_variant(pj.M2, pj.K);
      b.pjobs.push_back(pj);
      b.pack_max_cap = std::max(b.pack_max_cap, pj.cap);
    }
    pj.variant = -1;
    pj.packed += wide_offset(pj.M2, pj.K, pj.cap);
    b.pwjobs.push_back(pj);
    b.pack_wide_threads = std::max(b.pack_wide_threads, wide_pack_threads(pj.M2, pj.cap));
  }

  // detection tables sized for either kernel choice of every dual shape, so
  // that tuning can move jobs between the two launches in place
  size_t max_dj = 0, max_di = 0, max_wj = 0, max_wi = 0;
  for (const auto& it : b.items) {
    if (it.S <= 0) continue;
    if (detect_dual(it.model.M2, it.model.K)) {
      ++max_dj;
      max_di += detect_tiles(it.S);
    }
    ++max_wj;
    max_wi += wide_detect_items(it.S);
  }
  assign_detection(b);

  b.off_t = 0;
  b.off_rj = align256(b.off_t + b.tjobs.size() * sizeof(TrainJob));
  b.off_ri = align256(b.off_rj + b.rjobs.size() * sizeof(TrainJob));
  b.off_p = align256(b.off_ri + b.ritems.size() * sizeof(int4));
  b.off_pw = align256(b.off_p + b.pjobs.size() * sizeof(PackJob));
  b.off_d = align256(b.off_pw + b.pwjobs.size() * sizeof(PackJob));
  b.off_i = align256(b.off_d + max_dj * sizeof(DetJob));
  b.off_wd = align256(b.off_i + max_di * sizeof(int2));
  b.off_wi = align256(b.off_wd + max_wj * sizeof(DetJob));
  b.off_c = align256(b.off_wi + max_wi * sizeof(int2));
  b.off_rows = b.off_c + 256;                 // tables end here (the bound image)
  b.bytes = b.off_rows + b.rows_floats * sizeof(float);
  b.signature = signature_of(b.items);
  bool pers = true;
  if (tune_get_form(b.signature, &pers)) b.persistent = pers;
}

template <class T>
const T* at(const apsm_batch* b, size_t off) {
  return reinterpret_cast<const T*>(b->ws + off);
}

// The detection launches: split-FP16 (counter pair at off_c) and one
// two-contraction launch per padded width class c (pair at off_c + 8 + 8 c).
int run_detect(const apsm_batch* b, bool persistent, hipStream_t stream) {
  unsigned int* ctr = reinterpret_cast<unsigned int*>(b->ws + b->off_c);
  const int cus = b->cus > 0 && b->cus < b->grid ? b->cus : b->grid;
  for (int c = 0; c < 3; ++c) {
    const int n = b->wbegin[c + 1] - b->wbegin[c];
    if (n <= 0) continue;
    // workgroups per CU: two of the 32-wide specialisation, one of the wider
    hipError_t e = launch_detect_wide_batch(at<DetJob>(b, b->off_wd), at<int2>(b, b->off_wi) + b->wbegin[c], n,
                                            persistent ? ctr + 2 + 2 * c : nullptr, (c == 0 ? 2 : 1) * cus, c, stream);
    if (e != hipSuccess) return hip_status(e);
  }
  if (!b->ditems.empty()) {
    hipError_t e = launch_detect_batch(at<DetJob>(b, b->off_d), at<int2>(b, b->off_i), (int)b->ditems.size(),
                                       persistent ? ctr : nullptr, 2 * cus, stream);
    if (e != hipSuccess) return hip_status(e);
  }
  return APSM_OK;
}

}  // namespace

extern "C" {

int apsm_batch_create(const apsm_params_t* params, const apsm_batch_item_t* items, int n, apsm_batch_t** out) {
  if (!params || !items || !out || n < 1) return APSM_ERR_INVALID_ARG;
  *out = nullptr;
  apsm_params_t pc = *params;
  pc.sigma2 = 1.0f;                // per item
  pc.dict_cap = pc.window;         // per item
  if (int rc = check_params(&pc)) return rc;
  if (pc.init == APSM_INIT_CONTINUE) return APSM_ERR_UNSUPPORTED;   // kernel rows cover the pilots only
  if (pc.set_types) return APSM_ERR_UNSUPPORTED;                     // hyperslabs only
  for (int i = 0; i < n; ++i)
    if (int rc = check_item(items[i], params->window)) return rc;
  if (!buffers_disjoint(std::vector<apsm_batch_item_t>(items, items + n))) return APSM_ERR_INVALID_ARG;
  apsm_batch* b = new (std::nothrow) apsm_batch();
  if (!b) return APSM_ERR_INVALID_ARG;
  b->items.assign(items, items + n);
  plan(*b, &pc);
  if (b->ditems.size() > (size_t)INT32_MAX || b->witems.size() > (size_t)INT32_MAX) {
    delete b;
    return APSM_ERR_UNSUPPORTED;
  }
  *out = b;
  return APSM_OK;
}

size_t apsm_batch_workspace_bytes(const apsm_batch_t* b) { return b ? b->bytes : 0; }

int apsm_batch_bind(apsm_batch_t* b, void* workspace, size_t bytes, void* stream) {
  if (!b) return APSM_ERR_INVALID_ARG;
  if (!workspace || bytes < b->bytes || (reinterpret_cast<uintptr_t>(workspace) & 255)) return APSM_ERR_WORKSPACE;
  // the tables (the kernel rows after them are written on the device)
  std::vector<unsigned char> img(b->off_rows, 0);
  if (!b->tjobs.empty()) std::memcpy(img.data() + b->off_t, b->tjobs.data(), b->tjobs.size() * sizeof(TrainJob));
  if (!b->rjobs.empty()) {
    std::vector<TrainJob> rj = b->rjobs;
    float* rows = reinterpret_cast<float*>(static_cast<unsigned char*>(workspace) + b->off_rows);
    for (size_t q = 0; q < rj.size(); ++q) {
      rj[q].glag = rows + b->rows_off[q];
      rj[q].kw = rj[q].glag + (size_t)2 * rj[q].P * rj[q].cap;
    }
    std::memcpy(img.data() + b->off_rj, rj.data(), rj.size() * sizeof(TrainJob));
  }
  if (!b->ritems.empty()) std::memcpy(img.data() + b->off_ri, b->ritems.data(), b->ritems.size() * sizeof(int4));
  if (!b->pjobs.empty()) std::memcpy(img.data() + b->off_p, b->pjobs.data(), b->pjobs.size() * sizeof(PackJob));
  if (!b->pwjobs.empty()) std::memcpy(img.data() + b->off_pw, b->pwjobs.data(), b->pwjobs.size() * sizeof(PackJob));
  if (!b->djobs.empty()) std::memcpy(img.data() + b->off_d, b->djobs.data(), b->djobs.size() * sizeof(DetJob));
  if (!b->ditems.empty()) std::memcpy(img.data() + b->off_i, b->ditems.data(), b->ditems.size() * sizeof(int2));
  if (!b->wjobs.empty()) std::memcpy(img.data() + b->off_wd, b->wjobs.data(), b->wjobs.size() * sizeof(DetJob));
  if (!b->witems.empty()) std::memcpy(img.data() + b->off_wi, b->witems.data(), b->witems.size() * sizeof(int2));
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(workspace, img.data(), img.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_status(e);
  b->ws = static_cast<unsigned char*>(workspace);
  b->grid = device_cus();
  return APSM_OK;
}

int apsm_batch_kernel_rows(const apsm_batch_t* b, void* stream) {
  if (!b || !b->ws) return APSM_ERR_INVALID_ARG;
  return hip_status(launch_kernel_rows(at<TrainJob>(b, b->off_rj), at<int4>(b, b->off_ri), (int)b->ritems.size(),
                                       b->rows_max_m2, b->cm, (hipStream_t)stream));
}

int apsm_batch_train(const apsm_batch_t* b, void* stream) {
  if (int rc = apsm_batch_kernel_rows(b, stream)) return rc;
  return apsm_batch_train_prepared(b, stream);
}

int apsm_batch_train_prepared(const apsm_batch_t* b, void* stream) {
  if (!b || !b->ws) return APSM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_train_rows(at<TrainJob>(b, b->off_rj), (int)b->rjobs.size(), b->cm, b->rows_lds, s);
  if (e == hipSuccess) e = launch_train_table(at<TrainJob>(b, b->off_t), (int)b->tjobs.size(), b->cm, b->train_lds, s);
  for (size_t q = 0; q < b->train_plain.size() && e == hipSuccess; ++q) {
    // shapes outside the table kernel (2M > 64, dictionaries past the rows
    // form): one launch each
    const auto& it = b->items[b->train_plain[q]];
    TrainArgs a{};
    a.cm = b->cm;
    a.rx = it.rx_pilot;
    a.sym = it.sym_pilot;
    a.dict[0] = it.model.dict;
    a.alpha[0] = it.model.alpha;
    a.w[0] = it.model.w;
    a.state[0] = it.model.state;
    a.n_inst = 1;
    a.P = it.P;
    a.M2 = it.model.M2;
    a.K = it.model.K;
    a.cap = it.model.dict_cap;
    a.c2 = kLog2e / (2.0f * it.sigma2);
    e = launch_train(a, s);
  }
  // packing reads the trained models: after every training launch
  if (e == hipSuccess) e = launch_pack_model_batch(at<PackJob>(b, b->off_p), (int)b->pjobs.size(), b->pack_max_cap, s);
  if (e == hipSuccess)
    e = launch_pack_wide_batch(at<PackJob>(b, b->off_pw), (int)b->pwjobs.size(), b->pack_wide_threads, s);
  return hip_status(e);
}

int apsm_batch_detect(const apsm_batch_t* b, void* stream) {
  if (!b || !b->ws) return APSM_ERR_INVALID_ARG;
  return run_detect(b, b->persistent, (hipStream_t)stream);
}

int apsm_batch_tune(apsm_batch_t* b, void* stream) {
  if (!b || !b->ws) return APSM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (b->ditems.empty() && b->witems.empty()) return APSM_OK;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return hip_status(hipGetLastError());
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_status(hipGetLastError());
  }
  int rc = APSM_OK;
  // best of three timed runs after one warm-up
  auto time_ms = [&](auto&& run, float* best) {
    rc = run();
    for (int rep = 0; rep < 3 && rc == APSM_OK; ++rep) {
      hipError_t e = hipEventRecord(e0, s);
      if (e == hipSuccess) rc = run();
      if (rc == APSM_OK && e == hipSuccess) e = hipEventRecord(e1, s);
      if (rc == APSM_OK && e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (rc == APSM_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) rc = hip_status(e);
      if (rep == 0 || ms < *best) *best = ms;
    }
  };

  // 1. the detection kernel of every shape class both kernels hold (2M as the
  //    split-FP16 kernel pads it, K): both timed on the class's largest
  //    detector of this batch, the faster recorded in the tuning cache
  std::map<std::pair<int, int>, int> classes;       // (padded 2M, K) -> item
  for (int i = 0; i < (int)b->items.size(); ++i) {
    const auto& it = b->items[i];
    if (it.S <= 0 || !detect_dual(it.model.M2, it.model.K)) continue;
    const int m2p = it.model.M2 <= 16 ? 16 : it.model.M2 <= 32 ? 32 : 64;
    auto f = classes.find({m2p, it.model.K});
    if (f == classes.end() || b->items[f->second].S < it.S) classes[{m2p, it.model.K}] = i;
  }
  for (const auto& cl : classes) {
    if (rc != APSM_OK) break;
    const auto& it = b->items[cl.second];
    const DetectArgs a = detect_args(&it.model, it.sigma2, it.S, it.rx, it.soft, it.hard, it.modulation, it.truth,
                                     it.err_count);
    float t[2] = {0.0f, 0.0f};
    for (int k = 0; k < 2 && rc == APSM_OK; ++k)
      time_ms([&] { return hip_status(launch_detect_with(a, k == 0 ? kDetectF16 : kDetectWide, s)); }, &t[k]);
    if (rc == APSM_OK) tune_set_kernel(it.model.M2, it.model.K, t[0] < t[1] ? kDetectF16 : kDetectWide);
  }
  if (rc == APSM_OK && !classes.empty()) {
    // move the jobs to the launches of their chosen kernels (tables rewritten in place)
    assign_detection(*b);
    const std::pair<size_t, const void*> parts[4] = {
        {b->djobs.size() * sizeof(DetJob), b->djobs.data()}, {b->ditems.size() * sizeof(int2), b->ditems.data()},
        {b->wjobs.size() * sizeof(DetJob), b->wjobs.data()}, {b->witems.size() * sizeof(int2), b->witems.data()}};
    const size_t offs[4] = {b->off_d, b->off_i, b->off_wd, b->off_wi};
    for (int q = 0; q < 4 && rc == APSM_OK; ++q) {
      if (parts[q].first == 0) continue;
      hipError_t e = hipMemcpyAsync(b->ws + offs[q], parts[q].second, parts[q].first, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = hip_status(e);
    }
  }

  // 2. the launch form: persistent workgroups claiming items, or one
  //    workgroup per item
  float best[2] = {0.0f, 0.0f};
  for (int form = 0; form < 2 && rc == APSM_OK; ++form)
    time_ms([&] { return run_detect(b, form == 1, s); }, &best[form]);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != APSM_OK) return rc;
  b->persistent = best[1] <= best[0];
  tune_set_form(b->signature, b->persistent);
  return APSM_OK;
}

int apsm_batch_set_form(apsm_batch_t* b, int persistent, int cus) {
  if (!b) return APSM_ERR_INVALID_ARG;
  b->persistent = persistent != 0;
  b->cus = cus > 0 ? cus : 0;
  return APSM_OK;
}

void apsm_batch_destroy(apsm_batch_t* b) { delete b; }


}  // extern "C"
