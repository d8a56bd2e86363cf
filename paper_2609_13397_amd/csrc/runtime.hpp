// Host runtime pieces of the library: error reporting, scratch memory, profiling.
#pragma once

#include <cstddef>
#include <stdexcept>
#include <string>
#include <vector>

#include "cg_common.hpp"

namespace cg {

// Thrown inside the library, turned into a cg_status at the C boundary.
struct Error : std::runtime_error {
  cg_status status;
  Error(cg_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void set_last_error(const std::string& msg);

#define CG_HIP(expr)                                                                                  \
  do {                                                                                                \
    hipError_t _e = (expr);                                                                           \
    if (_e != hipSuccess)                                                                             \
      throw ::cg::Error(CG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));               \
  } while (0)

#define CG_CHECK_ARG(cond, msg)                                                                       \
  do {                                                                                                \
    if (!(cond)) throw ::cg::Error(CG_ERR_INVALID_ARG, msg);                                          \
  } while (0)

// Library-owned caching pool: blocks freed on a stream are reused only on the same
// stream (stream order makes that safe without events), best fit; the cache is
// returned to the device when it exceeds 64 GiB.
void* pool_alloc(size_t bytes, hipStream_t s);
void pool_free(void* p, hipStream_t s);
void pool_release_all();

// Guard bands (a debugging aid, off by default): while enabled, every buffer placed
// by a Carve is followed by kGuardBytes holding kGuardWord, written before the call's
// kernels run and compared after them; a changed word means some kernel wrote past
// the end of its buffer.  Mode 2 also overwrites one guard word from the host before
// the comparison, to show that the check reports it.
constexpr size_t kGuardBytes = 256;
constexpr uint32_t kGuardWord = 0xC3A5F00Du;
int guard_mode();
void add_guard_violations(int64_t n);

// The buffers of one allocation phase, laid out back to back in one block: each
// starts on a 256-byte boundary and has 16 bytes of slack after it (then its guard
// band, when guard bands are on).  add() records where to store a buffer's address;
// place() stores them all once the block exists.
class Carve {
 public:
  template <class T>
  void add(T** out, size_t n) {
    add_bytes(reinterpret_cast<void**>(out), n * sizeof(T));
  }
  void add_bytes(void** out, size_t bytes) {
    items_.push_back(Item{out, offset_});
    size_t end = offset_ + bytes + 16;
    if (guard_) {
      end = (end + 3) / 4 * 4;
      guards_.push_back(end);
      end += kGuardBytes;
    }
    offset_ = (end + 255) / 256 * 256;
  }
  size_t bytes() const { return offset_ == 0 ? 256 : offset_; }
  void place(void* base) const {
    for (const Item& it : items_) *it.out = static_cast<char*>(base) + it.offset;
  }
  // Offsets of the guard bands in the block (empty when guard bands are off).
  const std::vector<size_t>& guards() const { return guards_; }

 private:
  struct Item {
    void** out;
    size_t offset;
  };
  std::vector<Item> items_;
  std::vector<size_t> guards_;
  size_t offset_ = 0;
  bool guard_ = guard_mode() != 0;
};

// A caller-provided device region that stands in for every allocation of a call.
struct FixedRegion {
  void* base;
  size_t bytes;
};

// Scratch allocations of one call, from the caller's cg_allocator or the pool, or, with
// a FixedRegion, consecutive 256-byte aligned pieces of that region (nothing is
// allocated or freed; asking for more than it holds is an argument error).
class Scratch {
 public:
  Scratch(const cg_allocator* a, hipStream_t s, const FixedRegion* fixed = nullptr)
      : user_(a ? *a : cg_allocator{nullptr, nullptr, nullptr}), s_(s), fixed_(fixed ? *fixed : FixedRegion{}) {}
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  ~Scratch() { release(); }

  void* get(size_t bytes);
  template <class T>
  T* get_n(size_t n) {
    return static_cast<T*>(get(n * sizeof(T) + 16));
  }
  // One block for every buffer of `c` (one allocator call per phase); writes the
  // guard bands, if any.
  void get(const Carve& c);
  // Frees, in stream order, the block of the last get(const Carve&); its guard bands
  // are no longer checked.  Not with a FixedRegion.
  void release_last();
  // Compares every guard band written so far with its pattern (synchronises the
  // stream); throws CG_ERR_STATE if a word changed.  No-op without guard bands.
  void check_guards();
  // Hands ownership of every block allocated so far to `out` (which releases them
  // later with the same allocator and stream).
  void transfer(std::vector<void*>& out) {
    out.insert(out.end(), blocks_.begin(), blocks_.end());
    blocks_.clear();
  }
  void release();
  const cg_allocator& allocator() const { return user_; }
  hipStream_t stream() const { return s_; }

 private:
  cg_allocator user_;
  hipStream_t s_;
  FixedRegion fixed_;
  size_t fixed_used_ = 0;
  std::vector<void*> blocks_;
  std::vector<uint32_t*> guards_;
  size_t last_guards_ = 0;  // guards_ before the last get(const Carve&)
};

void free_block(const cg_allocator& a, void* p, hipStream_t s);

// RAII profiling bracket around a kernel launch.
struct ProfScope {
  int stage;
  hipStream_t s;
  ProfScope(int st, hipStream_t str) : stage(st), s(str) { prof_begin(stage, s); }
  ~ProfScope() { prof_end(stage, s); }
};

}  // namespace cg
