// mci_batch.hip -- uneven batches (many plans over ragged packed buffers in one call) and
// the variant autotuner with its JSON cache.  Host code only: every kernel it queues is a
// plan's own, either as merged persistent launches over job tables (the single-pass 1-D
// kernel, the real-mode line-transform path and the 2-D line passes) or, for plans on
// other variants, as the plan's own launches on lane streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <unistd.h>
#include <vector>

#include "mci_jobs.h"
#include "mci_plan.h"

using namespace mci;

namespace mci {
JobRecorder*& job_recorder() {
  static thread_local JobRecorder* r = nullptr;
  return r;
}
}  // namespace mci

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) return fail(MCI_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// ================================================================= autotune cache
namespace mci {

static std::string device_key(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + "x" + std::to_string(prop.multiProcessorCount);
}

std::string plan_tune_key(const mci_plan_s* p) {
  std::ostringstream k;
  k << device_key(p->device) << "|";
  if (p->dims == 2) {
    k << "2d|h" << p->d2.h << "|w" << p->d2.w << "|s" << p->d2.scale << "|c" << p->d2.channels << "|p" << p->prec
      << "|st" << p->store;
    return k.str();
  }
  const mci_plan_desc& d = p->d;
  k << "1d|M" << d.M << "|N" << d.N << "|n1_" << d.n1 << "|out" << d.n_out << "|io" << d.real_io << "|p" << p->prec
    << "|st" << p->store << "|ch";
  for (int m = 0; m < d.M; ++m) k << (m ? "," : "") << d.ch[m].kind << "." << d.ch[m].order;
  k << "|ops";
  for (int o = 0; o < d.n_ops; ++o) k << (o ? "," : "") << d.ops[o] << "." << d.op_orders[o];
  return k.str();
}

// The cache is a JSON document with one entry object per line:
//   {"version": 1, "entries": [
//   {"key": "...", "variant": 2, "batch": 4096, "ms": [..]},
//   ...]}
// Keys hold no quotes or backslashes, so an entry's key and variant are read by scanning.
static std::map<std::string, std::string> read_cache(const std::string& path) {
  std::map<std::string, std::string> out;
  std::ifstream f(path);
  std::string line;
  const std::string kk = "\"key\": \"";
  while (std::getline(f, line)) {
    const size_t a = line.find(kk);
    if (a == std::string::npos) continue;
    const size_t b = line.find('"', a + kk.size());
    if (b == std::string::npos) continue;
    std::string entry = line.substr(line.find('{'));
    while (!entry.empty() && (entry.back() == ',' || entry.back() == ' ' || entry.back() == '\r')) entry.pop_back();
    out[line.substr(a + kk.size(), b - a - kk.size())] = entry;
  }
  return out;
}

int tune_cache_lookup(const std::string& path, const std::string& key) {
  const auto m = read_cache(path);
  const auto it = m.find(key);
  if (it == m.end()) return -1;
  const std::string vk = "\"variant\": ";
  const size_t a = it->second.find(vk);
  if (a == std::string::npos) return -1;
  return std::atoi(it->second.c_str() + a + vk.size());
}

static bool write_cache(const std::string& path, const std::map<std::string, std::string>& m) {
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "{\"version\": 1, \"entries\": [\n";
    size_t i = 0;
    for (const auto& kv : m) f << kv.second << (++i < m.size() ? ",\n" : "\n");
    f << "]}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace mci

// ================================================================= uneven batch
struct BatchClass {
  mci_plan_s* plan = nullptr;
  int64_t count = 0;
  int64_t* d_offs = nullptr;   // [count][2] (in_off, out_off), device
  double cost = 0.0;           // estimated bytes moved
  int lane = 0;
  bool merged = false;         // runs inside the merged launches (else on its lane)
  size_t ws_off = 0;           // merged: its own workspace region, from the job-region start
};

// One merged launch: the jobs of one kernel template at one step of the launch sequences of
// the classes on one lane.  Device tables (inside the batch's one table allocation): the jobs'
// argument structs, their virtual grids and the prefix of their workgroup counts.
struct JobGroup {
  MergedFn launch = nullptr;
  int lane = 0;
  int level = 0;
  MergedLaunch m{};
};

struct mci_batch_s {
  int device = 0;
  int lanes = 1;
  std::vector<BatchClass> cls;
  std::vector<hipStream_t> streams;   // one per lane (lanes > 1)
  std::vector<hipEvent_t> joins;      // one per lane
  hipEvent_t fork = nullptr;
  int64_t in_elems = 0, out_elems = 0;
  std::vector<JobGroup> groups;       // merged launches, by lane, in queue order
  void* d_jobtab = nullptr;           // device tables of every group
  size_t job_ws = 0;                  // workspace bytes of the merged classes
};

static void destroy_batch(mci_batch_s* b) {
  if (!b) return;
  if (b->cls.empty()) {
    delete b;
    return;
  }
  (void)hipSetDevice(b->device);
  for (auto& c : b->cls)
    if (c.d_offs) (void)hipFree(c.d_offs);
  if (b->d_jobtab) (void)hipFree(b->d_jobtab);
  for (hipStream_t s : b->streams)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->joins)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

static size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

// Workspace: first the lanes' regions, each the largest need of its lane classes (they run
// one after another), then the merged classes' regions, one per class (every merged class
// is in flight at once).  lane_off: offsets of the lane regions; returns the total bytes
// (plus 256 for aligning the caller's pointer) and the start of the merged regions.
static size_t batch_layout(const mci_batch_s* b, std::vector<size_t>& lane_off, size_t* job_start = nullptr) {
  std::vector<size_t> need(b->lanes, 0);
  for (const auto& c : b->cls)
    if (!c.merged) need[c.lane] = std::max(need[c.lane], plan_workspace(c.plan, c.count));
  lane_off.assign(b->lanes, 0);
  size_t total = 0;
  for (int l = 0; l < b->lanes; ++l) {
    lane_off[l] = total;
    total += al256(need[l]);
  }
  if (job_start) *job_start = total;
  total += b->job_ws;
  return total ? total + 256 : 0;
}

// Record every merged class's launches (its plan's own kernels, with tagged input, output
// and workspace pointers) and build the merged launches: one per (lane, step, kernel
// template).  A lane runs its merged launches in step order on its own stream, so the
// classes of different lanes never wait for each other.
static mci_status build_merged(mci_batch_s* b) {
  std::vector<size_t> lane_off;
  size_t job_start = 0;
  (void)batch_layout(b, lane_off, &job_start);
  struct Rec {
    Job job;
    int lane, level;
  };
  std::vector<Rec> recs;
  for (const auto& c : b->cls) {
    if (!c.merged) continue;
    JobRecorder rec;
    job_recorder() = &rec;
    const mci_status st = plan_run(c.plan, (const void*)kTagIn, (void*)kTagOut, c.count,
                                   (void*)(kTagWs + job_start + c.ws_off), c.d_offs, nullptr);
    job_recorder() = nullptr;
    if (st != MCI_OK) return st;
    for (size_t k = 0; k < rec.jobs.size(); ++k) recs.push_back({std::move(rec.jobs[k]), c.lane, (int)k});
  }
  // groups in (lane, level, first appearance) order
  std::vector<std::vector<size_t>> members;
  for (size_t r = 0; r < recs.size(); ++r) {
    size_t g = 0;
    for (; g < b->groups.size(); ++g)
      if (b->groups[g].lane == recs[r].lane && b->groups[g].level == recs[r].level &&
          b->groups[g].launch == recs[r].job.launch)
        break;
    if (g == b->groups.size()) {
      JobGroup jg;
      jg.launch = recs[r].job.launch;
      jg.lane = recs[r].lane;
      jg.level = recs[r].level;
      b->groups.push_back(jg);
      members.emplace_back();
    }
    members[g].push_back(r);
  }
  std::vector<size_t> order(b->groups.size());
  for (size_t g = 0; g < order.size(); ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    const JobGroup &gx = b->groups[x], &gy = b->groups[y];
    return gx.lane != gy.lane ? gx.lane < gy.lane : gx.level < gy.level;
  });
  // one device allocation holds every group's tables
  std::vector<size_t> off_args(order.size()), off_grid(order.size()), off_first(order.size());
  size_t bytes = 0;
  for (size_t i = 0; i < order.size(); ++i) {
    const auto& mem = members[order[i]];
    off_args[i] = bytes;
    bytes = al256(bytes + mem.size() * recs[mem[0]].job.args.size());
    off_grid[i] = bytes;
    bytes = al256(bytes + mem.size() * sizeof(JobGrid));
    off_first[i] = bytes;
    bytes = al256(bytes + (mem.size() + 1) * sizeof(int64_t));
  }
  std::vector<unsigned char> host(bytes, 0);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) return fail(MCI_E_DEVICE, "device properties");
  if (bytes && hipMalloc(&b->d_jobtab, bytes) != hipSuccess) {
    b->d_jobtab = nullptr;
    return fail(MCI_E_OUT_OF_MEMORY, "job tables");
  }
  std::vector<JobGroup> sorted;
  for (size_t i = 0; i < order.size(); ++i) {
    JobGroup g = b->groups[order[i]];
    const auto& mem = members[order[i]];
    const size_t asz = recs[mem[0]].job.args.size();
    int64_t total = 0;
    size_t lds = 0;
    for (size_t k = 0; k < mem.size(); ++k) {
      const Job& j = recs[mem[k]].job;
      if (j.args.size() != asz) return fail(MCI_E_DEVICE, "job argument size mismatch");
      std::memcpy(host.data() + off_args[i] + k * asz, j.args.data(), asz);
      std::memcpy(host.data() + off_grid[i] + k * sizeof(JobGrid), &j.grid, sizeof(JobGrid));
      std::memcpy(host.data() + off_first[i] + k * sizeof(int64_t), &total, sizeof(int64_t));
      total += j.grid.gx * j.grid.gy;
      lds = std::max(lds, j.lds);
    }
    std::memcpy(host.data() + off_first[i] + mem.size() * sizeof(int64_t), &total, sizeof(int64_t));
    const Job& j0 = recs[mem[0]].job;
    const int64_t resident = (int64_t)j0.occupancy(lds) * prop.multiProcessorCount;
    char* base = (char*)b->d_jobtab;
    g.m.jobs = base + off_args[i];
    g.m.grids = (const JobGrid*)(base + off_grid[i]);
    g.m.first = (const int64_t*)(base + off_first[i]);
    g.m.n_jobs = (int)mem.size();
    g.m.total = total;
    g.m.grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(total, resident));
    g.m.lds = lds;
    sorted.push_back(g);
  }
  b->groups.swap(sorted);
  if (bytes && hipMemcpy(b->d_jobtab, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
    return fail(MCI_E_DEVICE, "job table upload");
  if (std::getenv("MCI_BATCH_DEBUG"))
    for (const auto& g : b->groups)
      std::fprintf(stderr, "[mci batch] lane %d step %d: %d jobs, %lld workgroups on a grid of %u, %zu B LDS\n",
                   g.lane, g.level, g.m.n_jobs, (long long)g.m.total, g.m.grid, g.m.lds);
  return MCI_OK;
}

// A class runs inside the merged launches when merging is asked for (MCI_BATCH_MERGED=1 at
// batch creation) and its plan's active kernels record as jobs.  Merging is not the default:
// on the mixed workload it measured 2.59 ms per batch against 2.23 ms for each class's own
// launches on the lanes (the merged kernels hold the job arguments in 20-30 more registers
// and wait at every step for the lane's slowest class).
static bool mergeable(const mci_plan_s* p) {
  const char* e = std::getenv("MCI_BATCH_MERGED");
  if (!e || std::strcmp(e, "1") != 0) return false;
  if (p->dims == 2) return p->lp;
  return p->use_fused || p->use_real;
}

extern "C" {

mci_status mci_batch_create(const mci_batch_item* items, int64_t n_items, int lanes, mci_batch_t* out) {
  if (!out) return fail(MCI_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_items < 0 || (n_items > 0 && !items)) return fail(MCI_E_INVALID_ARG, "bad item list");
  if (lanes < 0 || lanes > 16) return fail(MCI_E_INVALID_ARG, "lanes must be in 0..16");
  if (lanes == 0) lanes = 16;
  mci_batch_s* b = new (std::nothrow) mci_batch_s();
  if (!b) return fail(MCI_E_OUT_OF_MEMORY, "batch");
  std::map<mci_plan_s*, size_t> index;
  std::vector<std::vector<int64_t>> offs;
  std::vector<std::pair<int64_t, int64_t>> out_ranges;
  int store = -1;
  for (int64_t i = 0; i < n_items; ++i) {
    const mci_batch_item& it = items[i];
    mci_plan_s* p = it.plan;
    if (!p) { destroy_batch(b); return fail(MCI_E_INVALID_ARG, "item " + std::to_string(i) + ": NULL plan"); }
    if (store < 0) { store = p->store; b->device = p->device; }
    if (p->store != store || p->device != b->device) {
      destroy_batch(b);
      return fail(MCI_E_INVALID_ARG, "item " + std::to_string(i) + ": plans differ in device or element type");
    }
    if (it.in_off < 0 || it.out_off < 0 || it.in_off % 4 || it.out_off % 4) {
      destroy_batch(b);
      return fail(MCI_E_INVALID_ARG, "item " + std::to_string(i) + ": offsets must be >= 0 and multiples of 4");
    }
    const int64_t ni = instance_in_elems(p), no = instance_out_elems(p);
    if (it.in_off > ((int64_t)1 << 46) || it.out_off > ((int64_t)1 << 46)) {
      destroy_batch(b);
      return fail(MCI_E_INVALID_ARG, "item " + std::to_string(i) + ": offset out of range");
    }
    b->in_elems = std::max(b->in_elems, it.in_off + ni);
    b->out_elems = std::max(b->out_elems, it.out_off + no);
    out_ranges.push_back({it.out_off, it.out_off + no});
    auto f = index.find(p);
    if (f == index.end()) {
      f = index.emplace(p, b->cls.size()).first;
      BatchClass c;
      c.plan = p;
      b->cls.push_back(c);
      offs.emplace_back();
    }
    BatchClass& c = b->cls[f->second];
    ++c.count;
    c.cost += (double)(ni + no) * store_bytes(store);
    offs[f->second].push_back(it.in_off);
    offs[f->second].push_back(it.out_off);
  }
  std::sort(out_ranges.begin(), out_ranges.end());
  for (size_t i = 1; i < out_ranges.size(); ++i)
    if (out_ranges[i].first < out_ranges[i - 1].second) {
      destroy_batch(b);
      return fail(MCI_E_INVALID_ARG, "output extents overlap at element " + std::to_string(out_ranges[i].first));
    }
  if (b->cls.empty()) {   // nothing to run: no device resources
    *out = b;
    return MCI_OK;
  }
  if (hipSetDevice(b->device) != hipSuccess) { destroy_batch(b); return fail(MCI_E_DEVICE, "hipSetDevice"); }
  for (auto& c : b->cls) {
    c.merged = mergeable(c.plan);
    if (c.merged) {
      c.ws_off = b->job_ws;
      b->job_ws += al256(plan_workspace(c.plan, c.count));
    }
  }
  for (size_t k = 0; k < b->cls.size(); ++k) {
    BatchClass& c = b->cls[k];
    const size_t bytes = offs[k].size() * sizeof(int64_t);
    if (hipMalloc(&c.d_offs, bytes) != hipSuccess) { destroy_batch(b); return fail(MCI_E_OUT_OF_MEMORY, "offset table"); }
    if (hipMemcpy(c.d_offs, offs[k].data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
      destroy_batch(b);
      return fail(MCI_E_DEVICE, "offset table upload");
    }
  }
  // lanes: classes in decreasing cost, each to the lane with the least cost so far
  b->lanes = std::max(1, std::min<int>(lanes, (int)b->cls.size()));
  {
    std::vector<size_t> order(b->cls.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return b->cls[x].cost > b->cls[y].cost; });
    std::vector<double> load(b->lanes, 0.0);
    for (size_t k : order) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      b->cls[k].lane = l;
      load[l] += b->cls[k].cost;
    }
    // within a lane, the largest classes first
    std::vector<BatchClass> sorted;
    for (size_t k : order) sorted.push_back(b->cls[k]);
    b->cls.swap(sorted);
  }
  {
    const mci_status st = build_merged(b);
    if (st != MCI_OK) {
      destroy_batch(b);
      return st;
    }
  }
  if (b->lanes > 1) {
    b->streams.assign(b->lanes, nullptr);
    b->joins.assign(b->lanes, nullptr);
    for (int l = 0; l < b->lanes; ++l) {
      // default priority: the lanes only add concurrency
      if (hipStreamCreateWithFlags(&b->streams[l], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&b->joins[l], hipEventDisableTiming) != hipSuccess) {
        destroy_batch(b);
        return fail(MCI_E_DEVICE, "lane stream");
      }
    }
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
      destroy_batch(b);
      return fail(MCI_E_DEVICE, "fork event");
    }
  }
  *out = b;
  return MCI_OK;
}

mci_status mci_batch_destroy(mci_batch_t b) {
  destroy_batch(b);
  return MCI_OK;
}

mci_status mci_batch_sizes(mci_batch_t b, int64_t* in_elems, int64_t* out_elems, size_t* ws_bytes) {
  if (!b) return fail(MCI_E_INVALID_ARG, "NULL batch");
  std::vector<size_t> lo;
  if (in_elems) *in_elems = b->in_elems;
  if (out_elems) *out_elems = b->out_elems;
  if (ws_bytes) *ws_bytes = batch_layout(b, lo);
  return MCI_OK;
}

mci_status mci_reconstruct_batch(mci_batch_t b, const void* in, void* out, void* workspace, size_t ws_bytes,
                                 hipStream_t stream) {
  if (!b) return fail(MCI_E_INVALID_ARG, "NULL batch");
  if (b->cls.empty()) return MCI_OK;
  if (!in || !out) return fail(MCI_E_INVALID_ARG, "NULL data pointer");
  if (!aligned16(in) || !aligned16(out) || !aligned16(workspace))
    return fail(MCI_E_INVALID_ARG, "data pointers and workspace must be 16-byte aligned");
  std::vector<size_t> lane_off;
  const size_t need = batch_layout(b, lane_off);
  if (need && (!workspace || ws_bytes < need))
    return fail(MCI_E_INVALID_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
  HIP_TRY(hipSetDevice(b->device));
  char* base = (char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  // per lane: its classes' own launches, then its merged launches in step order
  const JobBases jb{(const char*)in, (char*)out, base};
  auto run_lane = [&](int lane, hipStream_t s) -> mci_status {
    for (const auto& c : b->cls) {
      if (c.merged || c.lane != lane) continue;
      const mci_status st = plan_run(c.plan, in, out, c.count, base + lane_off[c.lane], c.d_offs, s);
      if (st != MCI_OK) return st;
    }
    for (const auto& g : b->groups) {
      if (g.lane != lane) continue;
      const hipError_t e = g.launch(g.m, jb, s);
      if (e != hipSuccess) return fail(MCI_E_DEVICE, std::string("merged launch: ") + hipGetErrorString(e));
    }
    return MCI_OK;
  };
  if (b->lanes == 1) return run_lane(0, stream);
  HIP_TRY(hipEventRecord(b->fork, stream));
  for (int l = 0; l < b->lanes; ++l) HIP_TRY(hipStreamWaitEvent(b->streams[l], b->fork, 0));
  mci_status st = MCI_OK;
  for (int l = 0; l < b->lanes && st == MCI_OK; ++l) st = run_lane(l, b->streams[l]);
  // always join, so a failed call still leaves the caller's stream (or capture) well formed
  for (int l = 0; l < b->lanes; ++l) {
    HIP_TRY(hipEventRecord(b->joins[l], b->streams[l]));
    HIP_TRY(hipStreamWaitEvent(stream, b->joins[l], 0));
  }
  return st;
}

// ================================================================= autotuner
mci_status mci_plan_autotune(mci_plan_t p, int64_t batch, const char* cache_path, mci_tune_result* res) {
  if (!p || batch < 1) return fail(MCI_E_INVALID_ARG, "NULL plan or batch < 1");
  if (batch > ((int64_t)1 << 34) / std::max<int64_t>(instance_in_elems(p), instance_out_elems(p)))
    return fail(MCI_E_INVALID_ARG, "batch too large to tune");
  mci_tune_result r{};
  r.variant = p->variant;
  r.batch = batch;
  for (double& m : r.ms) m = -1.0;
  std::string path = cache_path ? cache_path : "";
  if (path.empty()) {
    const char* env = std::getenv("MCI_TUNE_CACHE");
    if (env) path = env;
  }
  const std::string key = plan_tune_key(p);
  const uint32_t mask = plan_variant_mask(p);
  if (!path.empty()) {
    const int v = tune_cache_lookup(path, key);
    if (v >= 0 && (mask >> v & 1u)) {
      mci_status st = plan_set_variant(p, v);
      if (st != MCI_OK) return st;
      r.variant = v;
      r.from_cache = 1;
      if (res) *res = r;
      return MCI_OK;
    }
  }
  HIP_TRY(hipSetDevice(p->device));
  const size_t eb = (size_t)store_bytes(p->store);
  size_t ws_max = 0;
  const int keep = p->variant;
  for (int v = 0; v < MCI_NUM_VARIANTS; ++v)
    if (mask >> v & 1u) {
      (void)plan_set_variant(p, v);
      ws_max = std::max(ws_max, plan_workspace(p, batch));
    }
  (void)plan_set_variant(p, keep);
  void *din = nullptr, *dout = nullptr, *dws = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (din) (void)hipFree(din);
    if (dout) (void)hipFree(dout);
    if (dws) (void)hipFree(dws);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
  };
  const size_t in_bytes = (size_t)batch * instance_in_elems(p) * eb, out_bytes = (size_t)batch * instance_out_elems(p) * eb;
  if (hipMalloc(&din, in_bytes) != hipSuccess || hipMalloc(&dout, out_bytes) != hipSuccess ||
      (ws_max && hipMalloc(&dws, ws_max) != hipSuccess)) {
    cleanup();
    return fail(MCI_E_OUT_OF_MEMORY, "autotune buffers");
  }
  if (hipMemset(din, 0, in_bytes) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(MCI_E_DEVICE, "autotune set-up");
  }
  int best = -1;
  for (int v = 0; v < MCI_NUM_VARIANTS; ++v) {
    if (!(mask >> v & 1u)) continue;
    mci_status st = plan_set_variant(p, v);
    float ms = 0.f;
    // two warm-up calls, then enough timed calls for about 20 ms (3 to 50)
    for (int w = 0; w < 2 && st == MCI_OK; ++w) st = plan_run(p, din, dout, batch, dws, nullptr, s);
    int reps = 1;
    if (st == MCI_OK && hipEventRecord(e0, s) == hipSuccess) {
      st = plan_run(p, din, dout, batch, dws, nullptr, s);
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        st = MCI_E_DEVICE;
      reps = std::max(3, std::min(50, (int)(20.0 / std::max(ms, 1e-3f))));
    }
    if (st == MCI_OK && hipEventRecord(e0, s) == hipSuccess) {
      for (int k = 0; k < reps && st == MCI_OK; ++k) st = plan_run(p, din, dout, batch, dws, nullptr, s);
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        st = MCI_E_DEVICE;
    }
    if (st != MCI_OK) {
      (void)hipStreamSynchronize(s);
      (void)plan_set_variant(p, keep);
      cleanup();
      return fail(MCI_E_DEVICE, "autotune: variant " + std::to_string(v) + " failed");
    }
    r.ms[v] = (double)ms / reps;
    if (best < 0 || r.ms[v] < r.ms[best]) best = v;
  }
  cleanup();
  mci_status st = plan_set_variant(p, best);
  if (st != MCI_OK) return st;
  r.variant = best;
  if (!path.empty()) {
    auto m = read_cache(path);
    std::ostringstream e;
    e << "{\"key\": \"" << key << "\", \"variant\": " << best << ", \"batch\": " << batch << ", \"ms\": [";
    for (int v = 0; v < MCI_NUM_VARIANTS; ++v) {
      char buf[32];
      std::snprintf(buf, sizeof buf, "%.6g", r.ms[v]);
      e << (v ? ", " : "") << buf;
    }
    e << "]}";
    m[key] = e.str();
    (void)write_cache(path, m);
  }
  if (res) *res = r;
  return MCI_OK;
}

}  // extern "C"
