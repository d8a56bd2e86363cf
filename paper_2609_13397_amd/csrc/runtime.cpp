// Error reporting, the scratch-memory pool and per-stage profiling.
#include <atomic>
#include "runtime.hpp"

#include <map>
#include <mutex>
#include <unordered_map>

namespace cg {

// ------------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

}  // namespace cg

extern "C" const char* cg_last_error(void) { return cg::g_last_error.c_str(); }

namespace cg {

// ------------------------------------------------------------------------ pool

namespace {

struct PoolBlock {
  size_t bytes;
  hipStream_t stream;
  int device;
};

std::mutex g_pool_mu;
std::multimap<size_t, std::pair<void*, PoolBlock>> g_pool_free;  // by size
std::unordered_map<void*, PoolBlock> g_pool_live;

size_t g_pool_cached = 0;                                        // bytes in g_pool_free
constexpr size_t kPoolCacheLimit = size_t(64) << 30;             // beyond it the cache is returned

size_t round_bytes(size_t b) {
  if (b <= (1u << 20)) {
    size_t r = 256;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t g = 2u << 20;
  return (b + g - 1) / g * g;
}

}  // namespace

void* pool_alloc(size_t bytes, hipStream_t s) {
  int dev = 0;
  CG_HIP(hipGetDevice(&dev));
  const size_t want = round_bytes(bytes);
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    // best fit: the smallest cached block of this stream that holds the request, however
    // much larger (it is held for one call only), so that calls of varying sizes reuse
    // the blocks they have rather than adding one for every size they ask for
    for (auto it = g_pool_free.lower_bound(want); it != g_pool_free.end(); ++it) {
      if (it->second.second.stream == s && it->second.second.device == dev) {
        void* p = it->second.first;
        g_pool_live[p] = it->second.second;
        g_pool_cached -= it->first;
        g_pool_free.erase(it);
        return p;
      }
    }
  }
  bool trim = false;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    trim = g_pool_cached > kPoolCacheLimit;
  }
  if (trim) pool_release_all();  // a bound on the cache; rare (synchronises the device)
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    // give cached blocks back and retry once
    (void)hipGetLastError();
    pool_release_all();
    e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(CG_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pool_live[p] = PoolBlock{want, s, dev};
  return p;
}

void pool_free(void* p, hipStream_t s) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pool_live.find(p);
  if (it == g_pool_live.end()) return;
  PoolBlock b = it->second;
  b.stream = s;
  g_pool_live.erase(it);
  g_pool_free.emplace(b.bytes, std::make_pair(p, b));
  g_pool_cached += b.bytes;
}

void pool_release_all() {
  std::multimap<size_t, std::pair<void*, PoolBlock>> blocks;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    blocks.swap(g_pool_free);
    g_pool_cached = 0;
  }
  if (blocks.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : blocks) (void)hipFree(kv.second.first);
}

void* Scratch::get(size_t bytes) {
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  if (fixed_.base) {
    const size_t need = fixed_used_ + (bytes + 255) / 256 * 256;
    if (need > fixed_.bytes)
      throw Error(CG_ERR_INVALID_ARG, "the call needs more than the " + std::to_string(fixed_.bytes) +
                                          " bytes of its fixed scratch region (" + std::to_string(need) +
                                          " bytes so far)");
    p = static_cast<char*>(fixed_.base) + fixed_used_;
    fixed_used_ = need;
    return p;
  }
  if (user_.alloc) {
    p = user_.alloc(user_.ctx, bytes, s_);
    if (!p) throw Error(CG_ERR_OUT_OF_MEMORY, "allocator callback failed for " + std::to_string(bytes) + " bytes");
  } else {
    p = pool_alloc(bytes, s_);
  }
  blocks_.push_back(p);
  return p;
}

void free_block(const cg_allocator& a, void* p, hipStream_t s) {
  if (!p) return;
  if (a.free) a.free(a.ctx, p, s);
  else if (!a.alloc) pool_free(p, s);
}

void Scratch::get(const Carve& c) {
  char* base = static_cast<char*>(get(c.bytes()));
  c.place(base);
  last_guards_ = guards_.size();
  for (size_t off : c.guards()) {
    uint32_t* g = reinterpret_cast<uint32_t*>(base + off);
    CG_HIP(launch_fill_u32(g, kGuardWord, kGuardBytes / 4, s_));
    guards_.push_back(g);
  }
}

void Scratch::check_guards() {
  if (guards_.empty()) return;
  if (guard_mode() == 2) CG_HIP(launch_fill_u32(guards_.front(), ~kGuardWord, 1, s_));
  uint32_t* bad = static_cast<uint32_t*>(get(16));
  CG_HIP(launch_fill_u32(bad, 0u, 1, s_));
  for (const uint32_t* g : guards_) CG_HIP(launch_guard_check(g, (int)(kGuardBytes / 4), kGuardWord, bad, s_));
  uint32_t host_bad = 0;
  CG_HIP(hipMemcpyAsync(&host_bad, bad, sizeof(host_bad), hipMemcpyDeviceToHost, s_));
  CG_HIP(hipStreamSynchronize(s_));
  if (host_bad) {
    add_guard_violations(host_bad);
    throw Error(CG_ERR_STATE, "scratch guard bands overwritten: " + std::to_string(host_bad) + " word(s) in " +
                                  std::to_string(guards_.size()) + " guard bands");
  }
}

void Scratch::release_last() {
  if (fixed_.base || blocks_.empty()) throw Error(CG_ERR_STATE, "no block to release");
  free_block(user_, blocks_.back(), s_);
  blocks_.pop_back();
  guards_.resize(last_guards_);
}

void Scratch::release() {
  for (void* p : blocks_) free_block(user_, p, s_);
  blocks_.clear();
}

// ------------------------------------------------------------------------ profiling

namespace {

const char* kStageNames[ST_NUM] = {"camera",     "preprocess", "bin_count",      "depth_sort", "scan",
                                   "bin_emit",   "sort",       "tile_ranges",    "render",     "bwd_render",
                                   "bwd_reduce", "bwd_preprocess", "bake_rho2", "valu_probe"};

struct Pending {
  int stage;
  hipEvent_t a, b;
};

std::mutex g_prof_mu;
uint32_t g_prof_mask = 0;  // bit i: stage i is bracketed

// split tile render thresholds (cg_set_tile_split)
constexpr int64_t kSplitMaxTiles = 2048, kSplitMinLongest = 2048;
std::atomic<int64_t> g_split_max_tiles{kSplitMaxTiles}, g_split_min_long{kSplitMinLongest}, g_split_len{0};
std::atomic<int> g_guard_mode{0};
std::atomic<int64_t> g_guard_violations{0};
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_event_pool;
double g_total_ms[ST_NUM];
int64_t g_launches[ST_NUM];
thread_local hipEvent_t t_open[ST_NUM];

hipEvent_t get_event() {
  hipEvent_t e = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_event_pool.empty()) {
      e = g_event_pool.back();
      g_event_pool.pop_back();
    }
  }
  if (!e) CG_HIP(hipEventCreate(&e));
  return e;
}

}  // namespace

int guard_mode() { return g_guard_mode.load(); }
void add_guard_violations(int64_t n) { g_guard_violations += n; }

SplitPolicy split_policy() { return SplitPolicy{g_split_max_tiles.load(), g_split_min_long.load(), g_split_len.load()}; }

void prof_begin(int stage, hipStream_t s) {
  if (!((g_prof_mask >> stage) & 1u)) return;
  hipEvent_t e = get_event();
  CG_HIP(hipEventRecord(e, s));
  t_open[stage] = e;
}

void prof_end(int stage, hipStream_t s) {
  if (!t_open[stage]) return;
  hipEvent_t e = get_event();
  CG_HIP(hipEventRecord(e, s));
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_pending.push_back(Pending{stage, t_open[stage], e});
  t_open[stage] = nullptr;
}

}  // namespace cg

extern "C" {

int cg_profile_num_stages(void) { return cg::ST_NUM; }

const char* cg_profile_stage_name(int stage) {
  return (stage >= 0 && stage < cg::ST_NUM) ? cg::kStageNames[stage] : "";
}

void cg_profile_enable(int on) { cg::g_prof_mask = on ? ~0u : 0u; }

void cg_profile_enable_stages(uint32_t mask) { cg::g_prof_mask = mask; }

void cg_set_tile_split(int64_t max_tiles, int64_t min_longest, int64_t seg_len) {
  cg::g_split_max_tiles = max_tiles > 0 ? max_tiles : cg::kSplitMaxTiles;
  cg::g_split_min_long = min_longest > 0 ? min_longest : cg::kSplitMinLongest;
  cg::g_split_len = seg_len > 0 ? seg_len : 0;
}

void cg_debug_set_scratch_guards(int32_t mode) { cg::g_guard_mode = (mode >= 0 && mode <= 2) ? mode : 0; }

int64_t cg_debug_guard_violations(void) { return cg::g_guard_violations.load(); }

cg_status cg_profile_collect(void) {
  std::vector<cg::Pending> pend;
  {
    std::lock_guard<std::mutex> lk(cg::g_prof_mu);
    pend.swap(cg::g_pending);
  }
  cg_status st = CG_OK;
  for (auto& p : pend) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) {
      st = CG_ERR_HIP;
      cg::set_last_error("profiling event failed");
      continue;
    }
    std::lock_guard<std::mutex> lk(cg::g_prof_mu);
    cg::g_total_ms[p.stage] += ms;
    cg::g_launches[p.stage] += 1;
    cg::g_event_pool.push_back(p.a);
    cg::g_event_pool.push_back(p.b);
  }
  return st;
}

void cg_profile_read(double* total_ms, int64_t* launches) {
  std::lock_guard<std::mutex> lk(cg::g_prof_mu);
  for (int i = 0; i < cg::ST_NUM; ++i) {
    if (total_ms) total_ms[i] = cg::g_total_ms[i];
    if (launches) launches[i] = cg::g_launches[i];
    cg::g_total_ms[i] = 0.0;
    cg::g_launches[i] = 0;
  }
}

cg_status cg_release_cached_memory(void) {
  cg::pool_release_all();
  return CG_OK;
}

}  // extern "C"
