// Batched pipeline over items of different sizes: one persistent delay-and-sum launch (work
// units drawn from a device counter, most expensive items first), then each item's envelope
// and log/scan-conversion epilogue, captured in a HIP graph; plus the autotuner that picks the
// persistent launch shape by timing graph replays.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "das.h"

namespace usbf {
int envelope_enqueue(const float* in, int64_t n_rows, int n, float* env, float* row_max, hipStream_t s);
int validate_scan(const usbf_scan* s);
}  // namespace usbf

using namespace usbf;

struct usbf_batch_plan {
  std::vector<usbf_batch_item> items;
  BatchItemDev* d_items = nullptr;
  int* d_counter = nullptr;
  float* d_frame = nullptr;  // per-item frame maxima for the log compression (64 floats each)
  int n_items = 0, total_units = 0, grid = 0;
  usbf_batch_shape shape{};
  size_t lds = 0;
  bool vec = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int kFrameSlot = 64;

void destroy(usbf_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_counter) (void)hipFree(p->d_counter);
  if (p->d_frame) (void)hipFree(p->d_frame);
  delete p;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  return std::string(prop.gcnArchName);
}

// signature of the batch: architecture + FNV-1a hash of every item's sizes, in order
std::string batch_key(const usbf_batch_item* items, int n) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= uint64_t((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(n);
  for (int i = 0; i < n; ++i) {
    mix(items[i].geom.n_el);
    mix(items[i].geom.n_lines);
    mix(items[i].geom.lines_per_tx);
    mix(items[i].rx.n_samples);
    mix(items[i].rx.n_depth);
  }
  char buf[64];
  snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
  std::string arch = arch_name();
  for (char& c : arch)
    if (c == '"' || c == '\\') c = '_';
  return arch + "/" + buf;
}

// The cache is a flat JSON object:
//   {"<key>": {"groups_per_cu": g, "cost_order": c, "multi_line_tile": t, "chunk_div": d, "ms": ms}, ...}
std::map<std::string, std::string> read_cache(const char* path) {
  std::map<std::string, std::string> m;
  if (!path) return m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    const size_t kend = s.find('"', pos + 1);
    if (kend == std::string::npos) break;
    const std::string key = s.substr(pos + 1, kend - pos - 1);
    const size_t ob = s.find('{', kend), cb = s.find('}', kend);
    if (ob == std::string::npos || cb == std::string::npos || ob > cb) break;
    m[key] = s.substr(ob, cb - ob + 1);
    pos = cb + 1;
  }
  return m;
}

int json_int(const std::string& obj, const char* name, int dflt) {
  const std::string k = std::string("\"") + name + "\"";
  const size_t p = obj.find(k);
  if (p == std::string::npos) return dflt;
  const size_t c = obj.find(':', p);
  if (c == std::string::npos) return dflt;
  return atoi(obj.c_str() + c + 1);
}

int write_cache(const char* path, const std::map<std::string, std::string>& m) {
  std::ofstream f(path, std::ios::trunc);
  if (!f) return fail(USBF_EINVAL, "cannot write tune cache %s", path);
  f << "{\n";
  size_t i = 0;
  for (const auto& kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++i < m.size() ? ",\n" : "\n");
  f << "}\n";
  return USBF_OK;
}

int check_shape(const usbf_batch_shape& s) {
  USBF_REQUIRE(s.groups_per_cu >= 1 && s.groups_per_cu <= 8, USBF_EINVAL, "groups_per_cu %d outside 1..8",
               s.groups_per_cu);
  USBF_REQUIRE(s.cost_order == 0 || s.cost_order == 1, USBF_EINVAL, "cost_order must be 0 or 1");
  USBF_REQUIRE(s.multi_line_tile == 1 || s.multi_line_tile == 4, USBF_EINVAL, "multi_line_tile must be 1 or 4");
  USBF_REQUIRE(s.chunk_div >= 1 && s.chunk_div <= 8, USBF_EINVAL, "chunk_div %d outside 1..8", s.chunk_div);
  return USBF_OK;
}

constexpr usbf_batch_shape kDefaultShape = {2, 1, 4, 1};

int make_plan(const usbf_batch_item* items, int n, const usbf_batch_shape& shape, usbf_batch_plan** out,
              hipStream_t user_stream) {
  (void)user_stream;
  USBF_REQUIRE(items && out, USBF_EINVAL, "null items or plan");
  USBF_REQUIRE(n >= 1 && n <= 65536, USBF_EINVAL, "n_items %d out of range", n);
  int st0 = check_shape(shape);
  if (st0) return st0;
  const int groups_per_cu = shape.groups_per_cu, cost_order = shape.cost_order;
  std::vector<BatchItemDev> dev(n);
  bool vec = true;
  int max_el[2] = {0, 0};  // largest element count among 1-line and 4-line items
  for (int i = 0; i < n; ++i) {
    const usbf_batch_item& it = items[i];
    DasArgs a;
    int st = make_das_args(&it.geom, &it.rx, &a);
    if (st) return fail(st, "item %d: %s", i, usbf_last_error_detail());
    USBF_REQUIRE(it.rf && it.lines && it.row_max && it.image, USBF_EINVAL, "item %d: null buffer", i);
    st = validate_scan(&it.scan);
    if (st) return fail(st, "item %d: %s", i, usbf_last_error_detail());
    USBF_REQUIRE(it.scan.n_depth == it.rx.n_depth, USBF_ESHAPE, "item %d: scan and receive depth counts differ", i);
    const int64_t scan_lines = int64_t(it.scan.n_u) * (it.scan.kind == 1 ? it.scan.n_v : 1);
    USBF_REQUIRE(scan_lines == it.geom.n_lines, USBF_ESHAPE, "item %d: scan covers %lld lines, geometry %d", i,
                 (long long)scan_lines, it.geom.n_lines);
    USBF_REQUIRE(envelope_length_ok(it.rx.n_depth), USBF_EUNSUPPORTED, "item %d: n_depth %d", i, it.rx.n_depth);
    USBF_REQUIRE(finite_pos(it.dyn_range_db), USBF_EINVAL, "item %d: dyn_range_db", i);
    vec = vec && (it.rx.n_samples % 4 == 0) && ((reinterpret_cast<uintptr_t>(it.rf) & 7) == 0);
    const int G = it.geom.lines_per_tx >= 4 ? shape.multi_line_tile : 1;
    max_el[G == 4] = std::max(max_el[G == 4], it.geom.n_el);
    st = batch_item_setup(a, G, shape.chunk_div, &dev[i]);
    if (st) return fail(st, "item %d: %s", i, usbf_last_error_detail());
    dev[i].rf = it.rf;
    dev[i].out = it.lines;
  }
  const size_t lds = persistent_lds_bytes(max_el[0], max_el[1]);
  USBF_REQUIRE(lds <= 160 * 1024, USBF_EUNSUPPORTED, "items with %d / %d elements (1- / 4-line tiles) exceed the tile LDS",
               max_el[0], max_el[1]);
  // unit order: most expensive units (most elements) first, stable
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  if (cost_order)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return dev[x].a.n_el > dev[y].a.n_el; });
  std::vector<BatchItemDev> table(n);
  int64_t units = 0;
  for (int k = 0; k < n; ++k) {
    table[k] = dev[order[k]];
    table[k].unit_begin = int(units);
    units += table[k].n_units;
  }
  USBF_REQUIRE(units < (int64_t(1) << 30), USBF_EUNSUPPORTED, "too many work units");

  usbf_batch_plan* p = new usbf_batch_plan();
  p->items.assign(items, items + n);
  p->n_items = n;
  p->total_units = int(units);
  p->shape = shape;
  p->lds = lds;
  p->vec = vec;
  int dev_id = 0, n_cu = 0;
  if (hipGetDevice(&dev_id) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess) {
    destroy(p);
    return fail(USBF_EDEVICE, "device query failed");
  }
  p->grid = std::max(1, std::min(n_cu * groups_per_cu, p->total_units));
  if (hipMalloc(&p->d_items, sizeof(BatchItemDev) * n) != hipSuccess ||
      hipMalloc(&p->d_counter, 256) != hipSuccess ||
      hipMalloc(&p->d_frame, sizeof(float) * kFrameSlot * n) != hipSuccess ||
      hipMemcpy(p->d_items, table.data(), sizeof(BatchItemDev) * n, hipMemcpyHostToDevice) != hipSuccess) {
    destroy(p);
    return fail(USBF_EDEVICE, "batch plan allocation failed");
  }
  // capture on a private stream (the caller's may be the legacy null stream)
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    destroy(p);
    return fail(USBF_EDEVICE, "stream creation failed");
  }
  int st = USBF_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = fail(USBF_EDEVICE, "capture");
  if (!st) st = launch_persistent(p->d_items, n, p->total_units, p->d_counter, vec, p->grid, lds, cs);
  for (int i = 0; i < n && !st; ++i) {
    const usbf_batch_item& it = items[i];
    st = envelope_enqueue(it.lines, it.geom.n_lines, it.rx.n_depth, it.lines, it.row_max, cs);
    if (!st)
      st = usbf_log_scan_convert(it.lines, it.row_max, 1, &it.scan, it.dyn_range_db, 0.0f, it.image,
                                 p->d_frame + size_t(kFrameSlot) * i, sizeof(float) * kFrameSlot, cs);
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  if (!st && ec != hipSuccess) st = fail(USBF_EDEVICE, "end capture: %s", hipGetErrorString(ec));
  p->graph = g;
  if (!st && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
    st = fail(USBF_EDEVICE, "graph instantiation failed");
  (void)hipStreamDestroy(cs);
  if (st) {
    destroy(p);
    return st;
  }
  *out = p;
  return USBF_OK;
}

}  // namespace

extern "C" int usbf_batch_plan_create(const usbf_batch_item* items, int32_t n_items, const char* tune_cache,
                                      usbf_batch_plan** plan, hipStream_t stream) {
  USBF_REQUIRE(items && plan, USBF_EINVAL, "null items or plan");
  USBF_REQUIRE(n_items >= 1, USBF_EINVAL, "empty batch");
  usbf_batch_shape shape = kDefaultShape;
  const auto cache = read_cache(tune_cache);
  const auto it = cache.find(batch_key(items, n_items));
  if (it != cache.end()) {
    shape.groups_per_cu = json_int(it->second, "groups_per_cu", shape.groups_per_cu);
    shape.cost_order = json_int(it->second, "cost_order", shape.cost_order);
    shape.multi_line_tile = json_int(it->second, "multi_line_tile", shape.multi_line_tile);
    shape.chunk_div = json_int(it->second, "chunk_div", shape.chunk_div);
    if (check_shape(shape)) return fail(USBF_EINVAL, "tune cache %s: invalid entry", tune_cache);
  }
  return make_plan(items, n_items, shape, plan, stream);
}

extern "C" int usbf_batch_run(usbf_batch_plan* plan, hipStream_t stream) {
  USBF_REQUIRE(plan && plan->exec, USBF_EINVAL, "null plan");
  const hipError_t e = hipGraphLaunch(plan->exec, stream);
  if (e != hipSuccess) return fail(USBF_EDEVICE, "graph launch: %s", hipGetErrorString(e));
  return USBF_OK;
}

extern "C" int usbf_batch_plan_destroy(usbf_batch_plan* plan) {
  destroy(plan);
  return USBF_OK;
}

extern "C" int usbf_batch_plan_create_shaped(const usbf_batch_item* items, int32_t n_items,
                                             const usbf_batch_shape* shape, usbf_batch_plan** plan,
                                             hipStream_t stream) {
  USBF_REQUIRE(items && plan && shape, USBF_EINVAL, "null items, shape or plan");
  USBF_REQUIRE(n_items >= 1, USBF_EINVAL, "empty batch");
  return make_plan(items, n_items, *shape, plan, stream);
}

extern "C" int usbf_batch_plan_shape(const usbf_batch_plan* plan, usbf_batch_shape* shape) {
  USBF_REQUIRE(plan && shape, USBF_EINVAL, "null argument");
  *shape = plan->shape;
  return USBF_OK;
}

extern "C" int usbf_autotune(const usbf_batch_item* items, int32_t n_items, const char* tune_cache,
                             hipStream_t stream) {
  USBF_REQUIRE(items && tune_cache, USBF_EINVAL, "null items or cache path");
  USBF_REQUIRE(n_items >= 1, USBF_EINVAL, "empty batch");
  bool any_multi = false;
  for (int i = 0; i < n_items; ++i) any_multi = any_multi || items[i].geom.lines_per_tx >= 4;
  std::vector<usbf_batch_shape> cands;
  for (int tile : {4, 1}) {
    if (tile == 1 && !any_multi) continue;  // the same plan as tile 4
    for (int div : {1, 2})
      for (int g = 1; g <= 4; ++g) cands.push_back({g, 1, tile, div});
  }
  float best_ms = 1e30f;
  usbf_batch_shape best = kDefaultShape;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(USBF_EDEVICE, "event creation failed");
  int st = USBF_OK;
  for (const usbf_batch_shape& c : cands) {
    usbf_batch_plan* p = nullptr;
    st = make_plan(items, n_items, c, &p, stream);
    if (st) break;
    for (int w = 0; w < 2 && !st; ++w) st = usbf_batch_run(p, stream);
    const int reps = 5;
    (void)hipEventRecord(e0, stream);
    for (int r = 0; r < reps && !st; ++r) st = usbf_batch_run(p, stream);
    (void)hipEventRecord(e1, stream);
    float ms = 0.0f;
    if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = fail(USBF_EDEVICE, "timing failed");
    destroy(p);
    if (st) break;
    if (ms / reps < best_ms) {
      best_ms = ms / reps;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  auto cache = read_cache(tune_cache);
  char val[200];
  snprintf(val, sizeof val,
           "{\"groups_per_cu\": %d, \"cost_order\": %d, \"multi_line_tile\": %d, \"chunk_div\": %d, \"ms\": %.4f}",
           best.groups_per_cu, best.cost_order, best.multi_line_tile, best.chunk_div, best_ms);
  cache[batch_key(items, n_items)] = val;
  return write_cache(tune_cache, cache);
}
