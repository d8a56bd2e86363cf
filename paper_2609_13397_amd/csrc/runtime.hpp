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
// stream (stream order makes that safe without events).
void* pool_alloc(size_t bytes, hipStream_t s);
void pool_free(void* p, hipStream_t s);
void pool_release_all();

// Scratch allocations of one call, from the caller's cg_allocator or the pool.
class Scratch {
 public:
  Scratch(const cg_allocator* a, hipStream_t s) : user_(a ? *a : cg_allocator{nullptr, nullptr, nullptr}), s_(s) {}
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  ~Scratch() { release(); }

  void* get(size_t bytes);
  template <class T>
  T* get_n(size_t n) {
    return static_cast<T*>(get(n * sizeof(T) + 16));
  }
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
  std::vector<void*> blocks_;
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
