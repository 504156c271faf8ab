// Host-side contraction engine: labelled device tensors and a planner that
// maps a two-operand contraction onto the batched MFMA contraction kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "kernels.h"

namespace ctm {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_CHECK(expr)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      throw ::ctm::Error(e_ == hipErrorOutOfMemory ? -2 : -3,                                     \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

enum { T_F64 = 0, T_F32 = 1 };
inline size_t type_size(int t) { return t == T_F64 ? 8 : 4; }

// A strided view of device memory with one character label per axis.
struct TRef {
  void* p = nullptr;
  int type = T_F64;
  std::vector<int64_t> dim, str;
  std::string lab;
  int64_t numel() const {
    int64_t n = 1;
    for (auto d : dim) n *= d;
    return n;
  }
};

TRef view(void* p, int type, const std::vector<int64_t>& dims, const std::string& lab);   // row-major
TRef relabel(const TRef& t, const std::string& lab);
// Split axis ``label`` (dimension a*b) into two axes (a major, b minor).
TRef split_axis(const TRef& t, char label, int64_t a, int64_t b, char lab_major, char lab_minor);

struct Tape;

// Stream-ordered device memory.  While a tape records, every allocation is
// registered with it and frees are deferred until the tape is cleared, so that
// the values a backward pass needs stay alive.
//
// Freed blocks are cached per size class and handed out again: all work of a
// Dev is queued on its one stream, so a block freed after the kernels that use
// it were queued may serve any later request on that stream.  (The
// stream-ordered allocator costs several microseconds of host time per call,
// and a sweep allocates thousands of workspaces.)  The cache goes back to the
// device pool when the Dev is destroyed, and before a request that the pool
// cannot otherwise satisfy: then the caches of every live Dev of the process
// are returned (the contexts of a process are used from one thread at a time)
// and the device is synchronised before the request is retried.
struct Dev {
  hipStream_t stream = nullptr;
  Tape* tape = nullptr;
  bool pool_ready = false;
  // Optional caller-provided arena: while set, every block is cut from it
  // (256-byte aligned, in request order) and frees are ignored; a request
  // beyond its end throws.  No device allocation is made meanwhile.
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  std::unordered_map<void*, size_t> live;                    // block -> size class
  std::unordered_map<size_t, std::vector<void*>> cached;     // size class -> free blocks
  // Optional caller allocator (ctm_set_allocator): while set, new blocks come
  // from it; every block goes back to the allocator that made it when the
  // cache is released.
  struct UserAlloc {
    void* (*alloc)(size_t bytes, void* stream, void* user) = nullptr;
    void (*free)(void* ptr, void* stream, void* user) = nullptr;
    void* user = nullptr;
  };
  UserAlloc ua;
  std::unordered_map<void*, UserAlloc> user_blocks;
  Dev();
  Dev(const Dev&) = delete;
  Dev& operator=(const Dev&) = delete;
  ~Dev();
  void* alloc(size_t bytes);   // take(), registered with a recording tape
  void free(void* p);          // give(), deferred while a tape records
  void* take(size_t bytes);    // a cached block of the size class, else a new one
  void give(void* p);          // back to the cache
  void release();              // cached blocks back to the device pool
};

// Work of a Dev confined to an arena for the lifetime of the scope.
struct ArenaScope {
  Dev* d;
  ArenaScope(Dev* dev, void* p, size_t bytes) : d(dev) {
    d->arena = (char*)p;
    d->arena_bytes = bytes;
    d->arena_used = 0;
  }
  ~ArenaScope() {
    d->arena = nullptr;
    d->arena_bytes = d->arena_used = 0;
  }
};

// Bytes of the split-K partial-sum workspace the contraction planner takes
// for a product with M x N outputs, a sum of length K over ``batch``
// matrices and elements of ``elem`` bytes (0 when it does not split K).
int64_t split_workspace_bytes(int64_t M, int64_t N, int64_t K, int64_t batch, size_t elem);

// Owning device buffer released on the stream.
struct DBuf {
  Dev* dev = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(Dev* d, size_t b) : dev(d), p(d->alloc(b)), bytes(b) {}
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : dev(o.dev), p(o.p), bytes(o.bytes) { o.p = nullptr; }
  DBuf& operator=(DBuf&& o) noexcept {
    reset();
    dev = o.dev; p = o.p; bytes = o.bytes; o.p = nullptr;
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (p && dev) dev->free(p);
    p = nullptr;
  }
};

// Temporary tensor with a contiguous row-major layout.
struct Tmp {
  DBuf buf;
  TRef t;
  Tmp() = default;
  Tmp(Dev* d, int type, const std::vector<int64_t>& dims, const std::string& lab) {
    int64_t n = 1;
    for (auto x : dims) n *= x;
    buf = DBuf(d, (size_t)std::max<int64_t>(n, 1) * type_size(type));
    t = view(buf.p, type, dims, lab);
  }
};

// C = alpha * contraction(A, B) (+ C if beta); labels shared by A and B and
// absent from C are summed, labels in all three are batched.  ``mode`` picks
// the matrix-core path for float tensors (ctmk::MODE_F32 or MODE_BF16).
void contract(Dev& dev, int mode, const TRef& C, const TRef& A, const TRef& B, double alpha = 1.0, int beta = 0,
              const double* colscale = nullptr);

// out (any strides) = in (any strides) for axes matched by label; converts type.
void copy_into(Dev& dev, const TRef& out, const TRef& in, bool accumulate = false);

// New contiguous tensor holding ``in`` with its axes in the order ``lab``.
Tmp permuted(Dev& dev, const TRef& in, const std::string& lab, int type = -1);

void fill(Dev& dev, const TRef& t, double v);   // t must be contiguous

// Reverse-mode tape over the engine's operations.  A contraction C = a A.B is
// recorded with its operand views; its adjoint is again a labelled
// contraction (Abar += a Cbar.B, Bbar += a A.Cbar).  Copies (with type
// conversion) map adjoints back by labels.  Operations with a hand-written
// derivative (projectors, normalisation, energy) are recorded as closures.
// Adjoints live in buffers that mirror the registered forward buffers byte
// for byte: the adjoint view of a forward view has the same strides at the
// same offset.  Pointers not registered with the tape are constants.
struct Tape {
  struct Buf {
    size_t bytes = 0;
    void* adj = nullptr;     // adjoint buffer (allocated on first use unless given)
    bool own = false;
  };
  struct Op {
    int kind = 0;            // 0 contract, 1 copy, 2 custom
    TRef a, b, c;
    double alpha = 1.0;
    int mode = 0;
    bool accumulate = false;
    std::function<void()> backward;
  };
  Dev* dev = nullptr;
  bool on = false;
  int paused = 0;
  std::map<uintptr_t, Buf> bufs;
  std::vector<Op> ops;
  std::vector<void*> retained;

  bool recording() const { return on && paused == 0; }
  void begin(Dev* d);
  // register a forward buffer; ``adj`` (optional) is an external adjoint buffer of the same size
  void reg(void* p, size_t bytes, void* adj = nullptr);
  bool has(const void* p) const;
  // adjoint view of forward view t (zero-initialised buffer on first use); requires has(t.p)
  TRef adj(const TRef& t);
  void* adj_ptr(const void* p);
  void custom(std::function<void()> f);
  void backward();
  // Reverse pass over the recorded operations [lo, hi) only; the tape stays
  // as recorded, so that the range can be run again with other seeds.
  void backward_range(size_t lo, size_t hi);
  // Zero every adjoint buffer the tape allocated itself (registered external
  // adjoints are left to their owner).
  void zero_own_adjoints();
  void clear();          // frees retained forward buffers and owned adjoints
};

struct TapePause {
  Tape* t;
  explicit TapePause(Dev& d) : t(d.tape) { if (t) ++t->paused; }
  ~TapePause() { if (t) --t->paused; }
};

// Launch counts, algorithmic flops and (while ``timing`` is on) HIP-event
// times of the timed kernel families: 0, 1, 2 = contraction kernel on the
// FP64, FP32 and BF16 matrix-core paths, 3 = block Jacobi rounds, 4 = QR
// panels.  Every timed launch is bracketed by a pair of events on its stream;
// ``collect_ms`` sums their times per family.
constexpr int N_FAMILIES = 5;
enum { FAM_JACOBI = 3, FAM_PANEL = 4 };
struct Counters {
  int64_t launches = 0;
  double flops = 0;
  bool timing = false;
  std::vector<hipEvent_t> pool;
  std::vector<int> pool_mode;       // family of each timed launch
  size_t used = 0;
  int64_t mode_launches[N_FAMILIES] = {0, 0, 0, 0, 0};
  double mode_flops[N_FAMILIES] = {0, 0, 0, 0, 0};
  void reset_timing();
  void record(hipStream_t s, int family);
  void collect_ms(double* ms_per_family);
  // bookkeeping of one launch of ``family`` with ``flops`` algorithmic flops
  void count(int family, double fl) {
    mode_launches[family]++;
    mode_flops[family] += fl;
  }
};
extern Counters g_counters;

}  // namespace ctm
