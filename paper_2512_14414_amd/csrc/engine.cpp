// Contraction planner: labelled tensors -> batched MFMA contraction kernel.
#include "engine.h"

#include <mutex>
#include <set>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>

namespace ctm {

Counters g_counters;

void Counters::reset_timing() {
  used = 0;
  launches = 0;
  flops = 0;
  for (int i = 0; i < N_FAMILIES; ++i) { mode_launches[i] = 0; mode_flops[i] = 0; }
}

void Counters::record(hipStream_t s, int mode) {
  if (used == pool.size()) {
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    pool.push_back(e);
    pool_mode.push_back(0);
  }
  pool_mode[used] = mode;
  HIP_CHECK(hipEventRecord(pool[used++], s));
}

void Counters::collect_ms(double* ms) {
  for (int i = 0; i < N_FAMILIES; ++i) ms[i] = 0;
  if (used) HIP_CHECK(hipEventSynchronize(pool[used - 1]));
  for (size_t i = 0; i + 1 < used; i += 2) {
    float t = 0;
    HIP_CHECK(hipEventElapsedTime(&t, pool[i], pool[i + 1]));
    ms[pool_mode[i]] += t;
  }
}

TRef view(void* p, int type, const std::vector<int64_t>& dims, const std::string& lab) {
  if (dims.size() != lab.size()) throw Error(-1, "view: labels do not match rank: " + lab);
  TRef t;
  t.p = p;
  t.type = type;
  t.dim = dims;
  t.str.assign(dims.size(), 1);
  for (int i = (int)dims.size() - 2; i >= 0; --i) t.str[i] = t.str[i + 1] * dims[i + 1];
  t.lab = lab;
  return t;
}

TRef relabel(const TRef& t, const std::string& lab) {
  if (lab.size() != t.lab.size()) throw Error(-1, "relabel: rank mismatch " + t.lab + " -> " + lab);
  TRef r = t;
  r.lab = lab;
  return r;
}

TRef split_axis(const TRef& t, char label, int64_t a, int64_t b, char lab_major, char lab_minor) {
  size_t i = t.lab.find(label);
  if (i == std::string::npos || t.dim[i] != a * b) throw Error(-1, std::string("split_axis: bad axis ") + label);
  TRef r;
  r.p = t.p;
  r.type = t.type;
  for (size_t j = 0; j < t.lab.size(); ++j) {
    if (j == i) {
      r.dim.push_back(a); r.str.push_back(t.str[j] * b); r.lab.push_back(lab_major);
      r.dim.push_back(b); r.str.push_back(t.str[j]); r.lab.push_back(lab_minor);
    } else {
      r.dim.push_back(t.dim[j]); r.str.push_back(t.str[j]); r.lab.push_back(t.lab[j]);
    }
  }
  return r;
}

// Freed blocks stay in the device's default memory pool across
// synchronisations (its release threshold raised to the maximum): a sweep
// allocates and frees its workspaces thousands of times, and with the
// default threshold of zero every synchronisation would hand them back to the
// driver.  Done once per device.
static void retain_pool_memory() {
  static std::mutex mu;
  static std::set<int> done;
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return;
  std::lock_guard<std::mutex> lock(mu);
  if (!done.insert(d).second) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, d) != hipSuccess) return;
  uint64_t threshold = UINT64_MAX;
  (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
}

// Size classes: multiples of 256 bytes up to 4 KiB, then 2^k and 3 * 2^(k-1)
// (at most a third of a block unused).
static size_t size_class(size_t b) {
  if (b <= 4096) return (b + 255) & ~(size_t)255;
  const size_t p = (size_t)1 << (63 - __builtin_clzll(b));
  if (b == p) return b;
  const size_t mid = p + (p >> 1);
  return b <= mid ? mid : 2 * p;
}

// Registry of the live Devs; never destroyed, so that a Dev outliving the
// library's static objects at process exit still finds it.
static std::mutex& devs_mu() {
  static std::mutex* m = new std::mutex();
  return *m;
}
static std::set<Dev*>& devs() {
  static std::set<Dev*>* s = new std::set<Dev*>();
  return *s;
}

Dev::Dev() {
  std::lock_guard<std::mutex> lock(devs_mu());
  devs().insert(this);
}

Dev::~Dev() {
  release();
  std::lock_guard<std::mutex> lock(devs_mu());
  devs().erase(this);
}

// Every cache of the process back to the pool (or to the caller allocator
// that made the block), then wait until the frees are done.  The device is
// synchronised first: a cached block may have been used last on another
// stream than the one it is freed on.
static void release_all_caches() {
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> lock(devs_mu());
    for (Dev* d : devs()) d->release();
  }
  (void)hipDeviceSynchronize();
}

void* Dev::take(size_t bytes) {
  if (arena) {
    const size_t off = (arena_used + 255) & ~(size_t)255;
    const size_t sz = bytes == 0 ? 8 : bytes;
    if (off > arena_bytes || sz > arena_bytes - off)
      throw Error(-2, "scratch arena exhausted: " + std::to_string(off + sz) + " bytes needed, " +
                          std::to_string(arena_bytes) + " available");
    arena_used = off + sz;
    return arena + off;
  }
  if (!pool_ready) {
    retain_pool_memory();
    pool_ready = true;
  }
  const size_t sz = size_class(bytes == 0 ? 8 : bytes);
  auto it = cached.find(sz);
  if (it != cached.end() && !it->second.empty()) {
    void* p = it->second.back();
    it->second.pop_back();
    live[p] = sz;
    return p;
  }
  void* p = nullptr;
  if (ua.alloc) {
    p = ua.alloc(sz, (void*)stream, ua.user);
    if (!p) {
      release_all_caches();
      p = ua.alloc(sz, (void*)stream, ua.user);
    }
    if (!p) throw Error(-2, "the caller's allocator returned no block of " + std::to_string(sz) + " bytes");
    user_blocks[p] = ua;
    live[p] = sz;
    return p;
  }
  hipError_t e = hipMallocAsync(&p, sz, stream);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    release_all_caches();
    e = hipMallocAsync(&p, sz, stream);
  }
  if (e != hipSuccess) throw Error(e == hipErrorOutOfMemory ? -2 : -3, std::string("hipMallocAsync: ") + hipGetErrorString(e));
  live[p] = sz;
  return p;
}

void Dev::give(void* p) {
  if (arena && (char*)p >= arena && (char*)p < arena + arena_bytes) return;   // arena blocks are not freed
  auto it = live.find(p);
  if (it == live.end()) {   // not from take(): straight back to the pool
    (void)hipFreeAsync(p, stream);
    return;
  }
  cached[it->second].push_back(p);
  live.erase(it);
}

void Dev::release() {
  for (auto& kv : cached)
    for (void* p : kv.second) {
      auto u = user_blocks.find(p);
      if (u != user_blocks.end()) {
        const UserAlloc a = u->second;
        user_blocks.erase(u);
        a.free(p, (void*)stream, a.user);
      } else {
        (void)hipFreeAsync(p, stream);
      }
    }
  cached.clear();
}

void* Dev::alloc(size_t bytes) {
  void* p = take(bytes);
  if (tape && tape->recording()) tape->reg(p, bytes);
  return p;
}

void Dev::free(void* p) {
  if (!p) return;
  if (tape && tape->on && tape->bufs.count((uintptr_t)p)) {
    tape->retained.push_back(p);
    return;
  }
  give(p);
}

// ---------------------------------------------------------------------------
void Tape::begin(Dev* d) {
  clear();
  dev = d;
  d->tape = this;
  on = true;
}

void Tape::reg(void* p, size_t bytes, void* adjp) {
  Buf b;
  b.bytes = bytes;
  b.adj = adjp;
  bufs[(uintptr_t)p] = b;
}

static std::map<uintptr_t, Tape::Buf>::iterator find_buf(std::map<uintptr_t, Tape::Buf>& m, const void* p) {
  uintptr_t a = (uintptr_t)p;
  auto it = m.upper_bound(a);
  if (it == m.begin()) return m.end();
  --it;
  if (a >= it->first + it->second.bytes) return m.end();
  return it;
}

bool Tape::has(const void* p) const {
  auto& m = const_cast<std::map<uintptr_t, Buf>&>(bufs);
  return find_buf(m, p) != m.end();
}

void* Tape::adj_ptr(const void* p) {
  auto it = find_buf(bufs, p);
  if (it == bufs.end()) throw Error(-1, "tape: adjoint of an unregistered buffer");
  Buf& b = it->second;
  if (!b.adj) {
    b.adj = dev->take(b.bytes);
    HIP_CHECK(hipMemsetAsync(b.adj, 0, b.bytes, dev->stream));
    b.own = true;
  }
  return (char*)b.adj + ((uintptr_t)p - it->first);
}

TRef Tape::adj(const TRef& t) {
  TRef r = t;
  r.p = adj_ptr(t.p);
  return r;
}

void Tape::custom(std::function<void()> f) {
  Op o;
  o.kind = 2;
  o.backward = std::move(f);
  ops.push_back(std::move(o));
}

void Tape::backward() { backward_range(0, ops.size()); }

void Tape::zero_own_adjoints() {
  for (auto& kv : bufs)
    if (kv.second.own && kv.second.adj) HIP_CHECK(hipMemsetAsync(kv.second.adj, 0, kv.second.bytes, dev->stream));
}

void Tape::backward_range(size_t lo, size_t hi) {
  bool was = on;
  on = false;
  if (hi > ops.size()) hi = ops.size();
  for (size_t i = hi; i-- > lo;) {
    Op& o = ops[i];
    if (o.kind == 0) {
      if (!has(o.c.p)) continue;
      TRef cb = adj(o.c);
      if (has(o.a.p)) contract(*dev, o.mode, adj(o.a), cb, o.b, o.alpha, 1);
      if (has(o.b.p)) contract(*dev, o.mode, adj(o.b), o.a, cb, o.alpha, 1);
    } else if (o.kind == 1) {
      if (has(o.c.p) && has(o.a.p)) copy_into(*dev, adj(o.a), adj(o.c), true);
    } else {
      o.backward();
    }
  }
  on = was;
}

void Tape::clear() {
  on = false;
  ops.clear();
  for (auto& kv : bufs)
    if (kv.second.own && kv.second.adj) dev->give(kv.second.adj);
  bufs.clear();
  for (void* p : retained) dev->give(p);
  retained.clear();
  if (dev) dev->tape = nullptr;
}

namespace {

struct Level {
  int64_t dim;
  int64_t s[3];   // strides in A, B, C
};

struct Group {
  std::vector<Level> lv;
  bool in[3];     // which operands carry this group
};

// Merge neighbouring levels (outer, inner) that are contiguous in every operand of the group.
void merge(Group& g) {
  std::vector<Level> out;
  for (const Level& l : g.lv) {
    if (!out.empty()) {
      Level& o = out.back();
      bool ok = true;
      for (int q = 0; q < 3; ++q)
        if (g.in[q] && o.s[q] != l.s[q] * l.dim) ok = false;
      if (ok) {
        o.dim *= l.dim;
        for (int q = 0; q < 3; ++q) o.s[q] = l.s[q];
        continue;
      }
    }
    out.push_back(l);
  }
  g.lv = out;
}

void fill_group(const Group& g, int64_t& total, int64_t& inner, int64_t* so, int64_t* si) {
  total = 1;
  for (auto& l : g.lv) total *= l.dim;
  for (int q = 0; q < 3; ++q) so[q] = si[q] = 0;
  if (g.lv.empty()) { inner = 1; return; }
  const Level& li = g.lv.back();
  inner = g.lv.size() == 1 ? total : li.dim;
  for (int q = 0; q < 3; ++q) si[q] = li.s[q];
  if (g.lv.size() == 2)
    for (int q = 0; q < 3; ++q) so[q] = g.lv[0].s[q];
}

struct Plan {
  Group b, m, n, k;
  bool ok() const { return b.lv.size() <= 2 && m.lv.size() <= 2 && n.lv.size() <= 2 && k.lv.size() <= 2; }
};

Plan make_plan(const TRef& C, const TRef& A, const TRef& B) {
  struct Info { int64_t dim = -1; int64_t s[3] = {0, 0, 0}; bool in[3] = {false, false, false}; };
  std::map<char, Info> info;
  const TRef* ops[3] = {&A, &B, &C};
  for (int q = 0; q < 3; ++q) {
    const TRef& t = *ops[q];
    for (size_t i = 0; i < t.lab.size(); ++i) {
      Info& f = info[t.lab[i]];
      if (f.in[q]) throw Error(-1, std::string("contract: repeated label ") + t.lab[i]);
      if (f.dim >= 0 && f.dim != t.dim[i])
        throw Error(-1, std::string("contract: dimension mismatch for label ") + t.lab[i] + " in " + A.lab + "," +
                            B.lab + "->" + C.lab);
      f.dim = t.dim[i];
      f.s[q] = t.str[i];
      f.in[q] = true;
    }
  }
  Plan P;
  auto add = [&](Group& g, char c) {
    const Info& f = info[c];
    if (f.dim == 1) return;
    Level l;
    l.dim = f.dim;
    for (int q = 0; q < 3; ++q) l.s[q] = f.s[q];
    g.lv.push_back(l);
  };
  P.b.in[0] = P.b.in[1] = P.b.in[2] = true;
  P.m.in[0] = true; P.m.in[1] = false; P.m.in[2] = true;
  P.n.in[0] = false; P.n.in[1] = true; P.n.in[2] = true;
  P.k.in[0] = true; P.k.in[1] = true; P.k.in[2] = false;
  for (char c : C.lab) {
    const Info& f = info[c];
    if (f.in[0] && f.in[1]) add(P.b, c);
    else if (f.in[0]) add(P.m, c);
    else if (f.in[1]) add(P.n, c);
    else if (f.dim != 1) throw Error(-1, std::string("contract: output label not in inputs: ") + c);
  }
  for (char c : A.lab) {
    const Info& f = info[c];
    if (f.in[1] && !f.in[2]) add(P.k, c);
    else if (!f.in[1] && !f.in[2] && f.dim != 1)
      throw Error(-1, std::string("contract: label only in the first operand: ") + c + " in " + A.lab + "," + B.lab +
                          "->" + C.lab);
  }
  for (char c : B.lab) {
    const Info& f = info[c];
    if (!f.in[0] && !f.in[2] && f.dim != 1)
      throw Error(-1, std::string("contract: label only in the second operand: ") + c);
  }
  merge(P.b);
  merge(P.m);
  merge(P.n);
  merge(P.k);
  return P;
}

// Whether a product with M x N outputs (per batch) and a sum of length K is
// split over K (few output tiles and a long sum), and into which chunks.
bool split_k(int64_t M, int64_t N, int64_t K, int64_t batch, int64_t& kchunk, int64_t& ksplit) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64) * batch;
  if (tiles >= 128 || K < 256) return false;
  const int64_t want = std::min<int64_t>((512 + tiles - 1) / tiles, K / 128);
  if (want <= 1) return false;
  kchunk = ((K + want - 1) / want + 31) / 32 * 32;
  ksplit = (K + kchunk - 1) / kchunk;
  return true;
}

void launch_plan(Dev& dev, int mode, const Plan& P, const TRef& C, const TRef& A, const TRef& B, double alpha,
                 int beta, const double* colscale) {
  ctmk::GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = A.p; g.B = B.p; g.C = C.p;
  int64_t so[3], si[3];
  fill_group(P.b, g.batch, g.b_in, so, si);
  g.a_b_o = so[0]; g.a_b_i = si[0]; g.b_b_o = so[1]; g.b_b_i = si[1]; g.c_b_o = so[2]; g.c_b_i = si[2];
  fill_group(P.m, g.M, g.m_in, so, si);
  g.a_m_o = so[0]; g.a_m_i = si[0]; g.c_m_o = so[2]; g.c_m_i = si[2];
  fill_group(P.n, g.N, g.n_in, so, si);
  g.b_n_o = so[1]; g.b_n_i = si[1]; g.c_n_o = so[2]; g.c_n_i = si[2];
  fill_group(P.k, g.K, g.k_in, so, si);
  g.a_k_o = so[0]; g.a_k_i = si[0]; g.b_k_o = so[1]; g.b_k_i = si[1];
  g.alpha = alpha;
  g.beta = beta;
  g.colscale = colscale;
  g.ksplit = 1;
  g.kchunk = g.K;
  g.work = nullptr;
  if (g.batch > 65535) throw Error(-1, "contract: batch too large");
  if (((g.M + 63) / 64) * ((g.N + 63) / 64) > 2147483647LL) throw Error(-1, "contract: too many tiles");
  if (g.K == 0) {   // empty sum
    if (!beta) fill(dev, C, 0.0);
    return;
  }
  const int km = A.type == T_F64 ? ctmk::MODE_F64 : mode;
  const double fl = 2.0 * (double)g.M * (double)g.N * (double)g.K * (double)g.batch;
  // few output tiles and a long sum: split K over more workgroups (partials in a workspace)
  DBuf work;
  if (split_k(g.M, g.N, g.K, g.batch, g.kchunk, g.ksplit)) {
    if (g.ksplit > 65535) throw Error(-1, "contract: K too long to split");
    work = DBuf(&dev, (size_t)g.ksplit * g.batch * g.M * g.N * type_size(C.type));
    g.work = work.p;
  }
  g_counters.launches++;
  g_counters.flops += fl;
  g_counters.count(km, fl);
  if (g_counters.timing) g_counters.record(dev.stream, km);
  HIP_CHECK(ctmk::launch_contract(km, g, dev.stream));
  if (g_counters.timing) g_counters.record(dev.stream, km);
}

}  // namespace

int64_t split_workspace_bytes(int64_t M, int64_t N, int64_t K, int64_t batch, size_t elem) {
  int64_t kchunk = 0, ksplit = 0;
  if (M < 1 || N < 1 || K < 1 || batch < 1 || !split_k(M, N, K, batch, kchunk, ksplit)) return 0;
  return ksplit * batch * M * N * (int64_t)elem;
}

void contract(Dev& dev, int mode, const TRef& C, const TRef& A, const TRef& B, double alpha, int beta,
              const double* colscale) {
  if (A.type != B.type || A.type != C.type) throw Error(-1, "contract: operand types differ");
  if (dev.tape && dev.tape->recording()) {
    if (colscale) throw Error(-1, "contract: a column scale cannot be recorded");
    Tape::Op o;
    o.kind = 0;
    o.a = A; o.b = B; o.c = C;
    o.alpha = alpha;
    o.mode = mode;
    dev.tape->ops.push_back(o);
  }
  TapePause pause(dev);
  Plan P = make_plan(C, A, B);
  if (P.ok()) {
    launch_plan(dev, mode, P, C, A, B, alpha, beta, colscale);
    return;
  }
  // Fall back: transpose the inputs to [batch, m, k] / [batch, k, n] and, if C
  // still needs more than two levels per group, go through a contiguous result.
  std::string bl, ml, nl, kl;
  for (char c : C.lab) {
    bool ia = A.lab.find(c) != std::string::npos, ib = B.lab.find(c) != std::string::npos;
    if (ia && ib) bl += c; else if (ia) ml += c; else if (ib) nl += c;
  }
  for (char c : A.lab)
    if (B.lab.find(c) != std::string::npos && C.lab.find(c) == std::string::npos) kl += c;
  Tmp a2 = permuted(dev, A, bl + ml + kl);
  Tmp b2 = permuted(dev, B, bl + kl + nl);
  P = make_plan(C, a2.t, b2.t);
  if (P.ok()) {
    launch_plan(dev, mode, P, C, a2.t, b2.t, alpha, beta, colscale);
    return;
  }
  std::vector<int64_t> cd;
  for (char c : bl + ml + nl) cd.push_back(C.dim[C.lab.find(c)]);
  Tmp c2(&dev, C.type, cd, bl + ml + nl);
  P = make_plan(c2.t, a2.t, b2.t);
  if (!P.ok()) throw Error(-1, "contract: no plan for " + A.lab + "," + B.lab + "->" + C.lab);
  launch_plan(dev, mode, P, c2.t, a2.t, b2.t, alpha, 0, colscale);
  copy_into(dev, C, c2.t, beta != 0);
}

void copy_into(Dev& dev, const TRef& out, const TRef& in, bool accumulate) {
  if (out.lab.size() != in.lab.size()) throw Error(-1, "copy_into: rank mismatch " + in.lab + " -> " + out.lab);
  if (dev.tape && dev.tape->recording()) {
    Tape::Op o;
    o.kind = 1;
    o.a = in; o.c = out;
    o.accumulate = accumulate;
    dev.tape->ops.push_back(o);
  }
  ctmk::PermArgs p;
  std::memset(&p, 0, sizeof(p));
  // iterate in the order of ``out``; drop size-1 axes
  int nd = 0;
  for (size_t i = 0; i < out.lab.size(); ++i) {
    size_t j = in.lab.find(out.lab[i]);
    if (j == std::string::npos) throw Error(-1, "copy_into: label missing " + in.lab + " -> " + out.lab);
    if (in.dim[j] != out.dim[i]) throw Error(-1, "copy_into: dimension mismatch");
    if (out.dim[i] == 1) continue;
    if (nd >= ctmk::PERM_MAX_DIMS) throw Error(-1, "copy_into: too many axes");
    p.dims[nd] = out.dim[i];
    p.out_strides[nd] = out.str[i];
    p.in_strides[nd] = in.str[j];
    ++nd;
  }
  p.ndim = nd;
  p.accumulate = accumulate ? 1 : 0;
  HIP_CHECK(ctmk::launch_permute(p, in.type, in.p, out.type, out.p, dev.stream));
}

Tmp permuted(Dev& dev, const TRef& in, const std::string& lab, int type) {
  TapePause pause(dev);
  std::vector<int64_t> d;
  for (char c : lab) {
    size_t j = in.lab.find(c);
    if (j == std::string::npos) throw Error(-1, "permuted: label missing");
    d.push_back(in.dim[j]);
  }
  Tmp t(&dev, type < 0 ? in.type : type, d, lab);
  copy_into(dev, t.t, in);
  return t;
}

void fill(Dev& dev, const TRef& t, double v) {
  HIP_CHECK(ctmk::launch_fill(t.type, t.p, v, t.numel(), dev.stream));
}

}  // namespace ctm
