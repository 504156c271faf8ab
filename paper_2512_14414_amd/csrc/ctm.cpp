// Nested single-layer CTMRG on one MI355X: context, moves, energy and C ABI.
//
// Method: arXiv:2512.14414, Sec. II C (multi-site CTMRG on the nested cell,
// Fig. CTMRG, Eqs. PQ and QRSVD), Sec. II B (nested network, Eq. XY; impurity
// tensors for local operators) and Eq. ExpH (energy).
//
// Frames.  The right, up and down moves are the left move of the lattice
// turned by two, one and three quarter turns counter-clockwise.  Environment
// legs are listed counter-clockwise around each site (see include/ctm.h), so
// a quarter turn maps the tensors C2, C3, C4, C1 and T2, T3, T4, T1 of a
// position onto C1, C2, C3, C4 and T1, T2, T3, T4 of the turned position
// without moving any data; only the site tensors are stored once per frame.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ctm.h"
#include "engine.h"
#include "kernels.h"
#include "opt_kernels.h"
#include "qr_kernels.h"

using namespace ctm;

namespace {

thread_local std::string g_init_error;

#define RB_CHECK(expr)                                                                                    \
  do {                                                                                                    \
    rocblas_status s_ = (expr);                                                                           \
    if (s_ != rocblas_status_success) throw Error(CTM_ESOLVER, std::string(#expr) + ": rocblas status " + \
                                                               std::to_string((int)s_));                  \
  } while (0)

struct SiteRef {
  void* p = nullptr;
  int64_t dim[4] = {0, 0, 0, 0};   // l, u, r, d
};

// Unique one-character labels for named bonds.
struct Labels {
  std::map<std::string, char> m;
  char next = 33;
  char operator()(const std::string& name) {
    auto it = m.find(name);
    if (it != m.end()) return it->second;
    if (next > 126) throw Error(CTM_EINVAL, "label pool exhausted");
    char c = next++;
    m[name] = c;
    return c;
  }
};

// Saved state of one row's projector block for the reverse pass.
struct ProjRow {
  int64_t kd = 0, mn = 0;
  std::shared_ptr<DBuf> N, S, Ur, Vr, s, w;   // N, S row-major mn x kd; Ur, Vr column-major mn x r
  void* Nadj = nullptr;                        // forward address of N and S (their adjoints are looked up)
  void* Sadj = nullptr;
  double* P = nullptr;                         // forward address of P_I and Q_I (kd x chi row-major)
  double* Q = nullptr;
};

// Projector block of one column step of a forward sweep that the reverse
// pass recomputes: the projectors of every row (as column_projectors writes
// them) and what the row's adjoint needs besides N and S (U_rho, V_rho, s, w).
struct ProjCacheStep {
  int rows = 0;
  int64_t maxkd = 0;
  DBuf P, Q;
  std::vector<ProjRow> saved;
};

}  // namespace

struct ctm_ctx {
  Dev dev;
  rocblas_handle blas = nullptr;
  int d = 0, D = 0, chi = 0, Lx = 0, Ly = 0, nt = 0, prec = 0, NY = 0, NX = 0;
  // 0: the nested network of K, B, X, Y sites on a 2Ly x 2Lx cell (Sec. II B);
  // 1: the double-layer network of reduced tensors a = sum_s A A* with legs of
  //    dimension D^2 on the Ly x Lx cell (Eq. Tred)
  int layout = 0;
  DBuf a_frames;                  // double layout: A of every tensor in every frame (legs rotated), d*D^4 each
  std::vector<int> pattern;
  int st = T_F64;                 // storage type of sites and environment
  int mode = ctmk::MODE_F64;      // matrix-core path of the sweep's contractions
  int est = T_F64;                // storage type of the energy's intermediates
  int emode = ctmk::MODE_F64;     // matrix-core path of the energy's contractions (and their adjoints)
  DBuf A64;                       // float64 copy of the site tensors
  DBuf site_buf;
  std::vector<SiteRef> frames[4];
  DBuf env;
  std::vector<int64_t> slot_off, slot_leg;
  int64_t env_elems = 0;
  double cutoff = 1e-10, eta = 1e-12;
  int check_finite = 1;
  int jacobi_max_sweeps = 40;
  bool jacobi_one_launch = true;   // all rounds of a Jacobi sweep in one launch (when the grid fits the device)
  bool jacobi_coop = true;         // launch that kernel cooperatively (co-residency guaranteed by the runtime)
  int svd_method = 0;              // projector SVD of sweeps that are not differentiated: 0 exact, 1 randomized
  int conv_env = 0;                // delta of ctm_sweep: 0 corner spectra, 1 largest change of the (gauge-fixed) entries
  int conv_rdm = 0;                // delta of ctm_sweep: largest change of the trace-normalised plaquette density matrices
  DBuf rdm_a, rdm_b;               // those of the previous and the current environment (conv_rdm)
  DBuf env_prev;                   // environment before the sweep (conv_env)
  // Checkpointed reverse pass: the forward sweeps that are recomputed keep
  // their projector blocks (pc_fill), and the recomputation takes them
  // instead of factorising again (pc_use, consumed in order from pc_pos);
  // the recomputed half systems, QR and SVD would give the same bits.
  int proj_cache = 1;
  std::vector<ProjCacheStep>* pc_fill = nullptr;
  std::vector<ProjCacheStep>* pc_use = nullptr;
  size_t pc_pos = 0;
  int rsvd_oversample = 8, rsvd_power = 2;
  uint64_t rsvd_seed = 0;
  int64_t sweep_capacity = -1;     // workgroups of that launch the device holds at once (-1: not yet asked)
  DBuf spec_prev, spec_cur, dscal;   // spectra and a few device scalars
  bool have_prev = false;
  DBuf rdm_buf;
  int n_rdm = 0;
  DBuf flag;                      // int flags: [0] non-finite, [1] failed solves, [2] empty cuts, [3] zero tensors
  std::string err;
  // Current storage of every environment tensor (position-major, 8 slots):
  // normally views of ``env``; while a tape records, every update goes to a
  // fresh buffer so that the values read before stay intact for the reverse pass.
  std::vector<void*> slot_ptr;
  Tape tape;
  // Second stream for the independent half of a column step (the odd rows:
  // half systems, their QR, their part of M) in sweeps that are not recorded;
  // it has its own allocator cache, and every fork from the main stream is
  // joined back before the main stream uses its results.
  Dev side;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int streams = 2;

  void fork() {
    HIP_CHECK(hipEventRecord(ev_fork, dev.stream));
    HIP_CHECK(hipStreamWaitEvent(side.stream, ev_fork, 0));
  }
  void join() {
    HIP_CHECK(hipEventRecord(ev_join, side.stream));
    HIP_CHECK(hipStreamWaitEvent(dev.stream, ev_join, 0));
  }

  int64_t max_leg() const { return layout ? (int64_t)D * D : (int64_t)D * d; }
  int ny(int f) const { return (f & 1) ? NX : NY; }
  int nx(int f) const { return (f & 1) ? NY : NX; }
  int kind(int I, int J) const { return (I & 1) * 2 + (J & 1); }   // 0 K, 1 Y, 2 X, 3 B
  void leg_dims(int I, int J, int64_t* l) const {
    if (layout) {
      l[0] = l[1] = l[2] = l[3] = (int64_t)D * D;
      return;
    }
    int64_t Dd = (int64_t)D * d;
    switch (kind(I, J)) {
      case 0: l[0] = D; l[1] = D; l[2] = Dd; l[3] = D; break;
      case 1: l[0] = Dd; l[1] = D; l[2] = D; l[3] = Dd; break;
      case 2: l[0] = D; l[1] = D; l[2] = D; l[3] = D; break;
      default: l[0] = D; l[1] = Dd; l[2] = D; l[3] = D; break;
    }
  }
  // frame-f position -> frame-0 position
  void to_orig(int f, int I, int J, int& oi, int& oj) const {
    int rows = ny(f);
    for (int t = 0; t < f; ++t) {
      int i = J, j = rows - 1 - I;
      I = i; J = j;
      rows = (rows == NY) ? NX : NY;   // rows of the previous frame
    }
    oi = I; oj = J;
  }
  SiteRef site(int f, int I, int J) const {
    int a = ny(f), b = nx(f);
    I = ((I % a) + a) % a; J = ((J % b) + b) % b;
    return frames[f][(size_t)I * b + J];
  }
  TRef site_t(int f, int I, int J, const std::string& lab) const {
    SiteRef s = site(f, I, J);
    return view(s.p, st, {s.dim[0], s.dim[1], s.dim[2], s.dim[3]}, lab);
  }
  // environment tensor ``slot`` (0..3 = C1..C4, 4..7 = T1..T4) of frame-f position (I, J)
  TRef slot(int f, int I, int J, int k, const std::string& lab) const {
    int a = ny(f), b = nx(f);
    I = ((I % a) + a) % a; J = ((J % b) + b) % b;
    int oi, oj;
    to_orig(f, I, J, oi, oj);
    int ok = ((k & 3) + f) % 4 + (k & 4);
    size_t idx = ((size_t)oi * NX + oj) * 8 + ok;
    char* base = (char*)slot_ptr[idx];
    if (k < 4) return view(base, st, {chi, chi}, lab);
    return view(base, st, {chi, slot_leg[idx], chi}, lab);
  }
  size_t slot_index(int f, int I, int J, int k) const {
    int a = ny(f), b = nx(f);
    I = ((I % a) + a) % a; J = ((J % b) + b) % b;
    int oi, oj;
    to_orig(f, I, J, oi, oj);
    return ((size_t)oi * NX + oj) * 8 + ((k & 3) + f) % 4 + (k & 4);
  }
  int64_t slot_elems(size_t idx) const { return idx % 8 < 4 ? (int64_t)chi * chi : (int64_t)chi * slot_leg[idx] * chi; }
  void reset_slot_ptrs() {
    slot_ptr.resize(slot_off.size());
    for (size_t i = 0; i < slot_off.size(); ++i) slot_ptr[i] = (char*)env.p + slot_off[i] * type_size(st);
  }
  // Destination of an updated environment tensor: in place, or a fresh
  // buffer while the tape records.
  TRef out_slot(int f, int I, int J, int k, const std::string& lab) {
    if (tape.recording()) {
      size_t idx = slot_index(f, I, J, k);
      void* p = dev.alloc((size_t)slot_elems(idx) * type_size(st));
      tape.retained.push_back(p);
      slot_ptr[idx] = p;
    }
    return slot(f, I, J, k, lab);
  }
};

namespace {

void build_layout(ctm_ctx* c) {
  c->slot_off.assign((size_t)c->NY * c->NX * 8, 0);
  c->slot_leg.assign((size_t)c->NY * c->NX * 8, 0);
  int64_t off = 0;
  for (int I = 0; I < c->NY; ++I)
    for (int J = 0; J < c->NX; ++J) {
      int64_t l[4];
      c->leg_dims(I, J, l);
      const int64_t tleg[4] = {l[1], l[2], l[3], l[0]};   // T1 up, T2 right, T3 down, T4 left
      for (int k = 0; k < 8; ++k) {
        size_t idx = ((size_t)I * c->NX + J) * 8 + k;
        c->slot_off[idx] = off;
        if (k < 4) off += (int64_t)c->chi * c->chi;
        else {
          c->slot_leg[idx] = tleg[k - 4];
          off += (int64_t)c->chi * tleg[k - 4] * c->chi;
        }
      }
    }
  c->env_elems = off;
}

// Reduced tensors a_t[(l l'), (u u'), (r r'), (d d')] = sum_s A_t[s,l,u,r,d] A_t[s,l',u',r',d']
// (Eq. Tred; real tensors, fused legs ket index major) of every frame.
void build_sites_double(ctm_ctx* c) {
  Dev& dev = c->dev;
  const int d = c->d, D = c->D;
  const int64_t D2 = (int64_t)D * D, na = D2 * D2 * D2 * D2, nk = (int64_t)d * D * D * D * D;
  const size_t es = type_size(c->st);
  if (!c->site_buf.p) c->site_buf = DBuf(&dev, (size_t)(4 * c->nt * na) * es);
  const std::string lurd = "lurd";
  Tmp a8(&dev, T_F64, {D, D, D, D, D, D, D, D}, "lLuUrRdD");
  for (int t = 0; t < c->nt; ++t) {
    double* At = (double*)c->A64.p + t * nk;
    contract(dev, ctmk::MODE_F64, a8.t, view(At, T_F64, {d, D, D, D, D}, "slurd"),
             view(At, T_F64, {d, D, D, D, D}, "sLURD"));
    for (int f = 0; f < 4; ++f) {
      std::string rl;
      for (int i = 0; i < 4; ++i) rl += lurd[(i + f) % 4];   // new axis i = old axis (i+f) mod 4
      void* dst = (char*)c->site_buf.p + (size_t)(f * c->nt + t) * na * es;
      copy_into(dev, view(dst, c->st, {D2, D2, D2, D2}, rl), view(a8.buf.p, T_F64, {D2, D2, D2, D2}, lurd));
    }
  }
  // the site tensors themselves per frame (legs rotated like the reduced
  // tensors', physical index first), for the layered absorption of the sweep
  if (!c->a_frames.p) c->a_frames = DBuf(&dev, (size_t)(4 * c->nt * nk) * es);
  for (int t = 0; t < c->nt; ++t) {
    double* At = (double*)c->A64.p + t * nk;
    for (int f = 0; f < 4; ++f) {
      std::string rl = "s";
      for (int i = 0; i < 4; ++i) rl += lurd[(i + f) % 4];
      void* dst = (char*)c->a_frames.p + (size_t)(f * c->nt + t) * nk * es;
      copy_into(dev, view(dst, c->st, {d, D, D, D, D}, rl), view(At, T_F64, {d, D, D, D, D}, "slurd"));
    }
  }
  for (int f = 0; f < 4; ++f) {
    int a = c->ny(f), b = c->nx(f);
    c->frames[f].assign((size_t)a * b, SiteRef());
    for (int I = 0; I < a; ++I)
      for (int J = 0; J < b; ++J) {
        int oi, oj;
        c->to_orig(f, I, J, oi, oj);
        int t = c->pattern[(size_t)oi * c->Lx + oj];
        SiteRef s;
        s.p = (char*)c->site_buf.p + (size_t)(f * c->nt + t) * na * es;
        for (int q = 0; q < 4; ++q) s.dim[q] = D2;
        c->frames[f][(size_t)I * b + J] = s;
      }
  }
}

// Dense nested sites of every frame from the float64 site tensors.
void build_sites(ctm_ctx* c) {
  if (c->layout) {
    build_sites_double(c);
    return;
  }
  Dev& dev = c->dev;
  const int d = c->d, D = c->D;
  const int64_t Dd = (int64_t)D * d, n4 = (int64_t)D * D * D * D;
  // host-built delta tensors X[l,u,r,d] = d(l,r) d(u,d) and Y[(l,s),u,r,(d,s')] = d(l,r) d(u,d) d(s,s')
  std::vector<double> X(n4, 0.0), Y((size_t)Dd * D * D * Dd, 0.0);
  for (int l = 0; l < D; ++l)
    for (int u = 0; u < D; ++u) X[((size_t)(l * D + u) * D + l) * D + u] = 1.0;
  for (int l = 0; l < D; ++l)
    for (int s = 0; s < d; ++s)
      for (int u = 0; u < D; ++u) {
        int64_t li = (int64_t)l * d + s, di = (int64_t)u * d + s;
        Y[((size_t)(li * D + u) * D + l) * Dd + di] = 1.0;
      }
  DBuf xy(&dev, (X.size() + Y.size()) * 8);
  HIP_CHECK(hipMemcpyAsync(xy.p, X.data(), X.size() * 8, hipMemcpyHostToDevice, dev.stream));
  HIP_CHECK(hipMemcpyAsync((double*)xy.p + X.size(), Y.data(), Y.size() * 8, hipMemcpyHostToDevice, dev.stream));
  TRef Xt = view(xy.p, T_F64, {D, D, D, D}, "lurd");
  TRef Yt = view((double*)xy.p + X.size(), T_F64, {Dd, D, D, Dd}, "lurd");

  // per frame: K_t, B_t for each tensor, X, Y  (each d*D^4 or D^4 or d^2 D^4 elements)
  const int64_t nk = (int64_t)d * n4, ny_ = (int64_t)d * d * n4;
  const int64_t per_frame = 2 * c->nt * nk + n4 + ny_;
  if (!c->site_buf.p) c->site_buf = DBuf(&dev, (size_t)(4 * per_frame) * type_size(c->st));
  char* base = (char*)c->site_buf.p;
  const size_t es = type_size(c->st);
  const std::string lurd = "lurd";
  for (int f = 0; f < 4; ++f) {
    std::string rl;
    for (int i = 0; i < 4; ++i) rl += lurd[(i + f) % 4];   // new axis i = old axis (i+f) mod 4
    auto rot_dims = [&](const int64_t* od, int64_t* nd) {
      for (int i = 0; i < 4; ++i) nd[i] = od[(i + f) % 4];
    };
    char* fb = base + (size_t)f * per_frame * es;
    std::vector<SiteRef> K(c->nt), B(c->nt);
    SiteRef Xr, Yr;
    for (int t = 0; t < c->nt; ++t) {
      TRef At = view((double*)c->A64.p + t * nk, T_F64, {d, D, D, D, D}, "slurd");
      // K[l,u,(r s),d] and B[l,(u s),r,d]
      int64_t kd0[4] = {D, D, Dd, D}, bd0[4] = {D, Dd, D, D}, nd[4];
      // K in frame 0 as a 5-axis view over a temporary, then rotated
      Tmp k0(&dev, T_F64, {D, D, D, d, D}, "lursd");
      copy_into(dev, k0.t, At);
      Tmp b0(&dev, T_F64, {D, D, d, D, D}, "lusrd");
      copy_into(dev, b0.t, At);
      rot_dims(kd0, nd);
      K[t].p = fb + (size_t)(2 * t) * nk * es;
      std::memcpy(K[t].dim, nd, sizeof(nd));
      copy_into(dev, view(K[t].p, c->st, {nd[0], nd[1], nd[2], nd[3]}, rl),
                view(k0.buf.p, T_F64, {kd0[0], kd0[1], kd0[2], kd0[3]}, lurd));
      rot_dims(bd0, nd);
      B[t].p = fb + (size_t)(2 * t + 1) * nk * es;
      std::memcpy(B[t].dim, nd, sizeof(nd));
      copy_into(dev, view(B[t].p, c->st, {nd[0], nd[1], nd[2], nd[3]}, rl),
                view(b0.buf.p, T_F64, {bd0[0], bd0[1], bd0[2], bd0[3]}, lurd));
    }
    {
      int64_t xd0[4] = {D, D, D, D}, yd0[4] = {Dd, D, D, Dd}, nd[4];
      rot_dims(xd0, nd);
      Xr.p = fb + (size_t)(2 * c->nt) * nk * es;
      std::memcpy(Xr.dim, nd, sizeof(nd));
      copy_into(dev, view(Xr.p, c->st, {nd[0], nd[1], nd[2], nd[3]}, rl), Xt);
      rot_dims(yd0, nd);
      Yr.p = fb + ((size_t)(2 * c->nt) * nk + n4) * es;
      std::memcpy(Yr.dim, nd, sizeof(nd));
      copy_into(dev, view(Yr.p, c->st, {nd[0], nd[1], nd[2], nd[3]}, rl), Yt);
    }
    int a = c->ny(f), b = c->nx(f);
    c->frames[f].assign((size_t)a * b, SiteRef());
    for (int I = 0; I < a; ++I)
      for (int J = 0; J < b; ++J) {
        int oi, oj;
        c->to_orig(f, I, J, oi, oj);
        int t = c->pattern[(size_t)(oi / 2) * c->Lx + (oj / 2)];
        SiteRef s;
        switch (c->kind(oi, oj)) {
          case 0: s = K[t]; break;
          case 1: s = Yr; break;
          case 2: s = Xr; break;
          default: s = B[t]; break;
        }
        c->frames[f][(size_t)I * b + J] = s;
      }
  }
}

// Sites-derived starting environment (frame 0): each tensor is the nested
// neighbour with its outward legs summed over all indices.
void init_env(ctm_ctx* c) {
  Dev& dev = c->dev;
  fill(dev, view(c->env.p, c->st, {c->env_elems}, "e"), 0.0);
  int64_t mx = c->max_leg();
  Tmp ones(&dev, c->st, {mx, mx}, "pq");
  fill(dev, ones.t, 1.0);
  for (int I = 0; I < c->NY; ++I)
    for (int J = 0; J < c->NX; ++J) {
      auto nb = [&](int di, int dj, const std::string& lab) { return c->site_t(0, I + di, J + dj, lab); };
      auto one = [&](const TRef& s, const std::string& which) {
        std::vector<int64_t> dd;
        for (char ch : which) dd.push_back(s.dim[s.lab.find(ch)]);
        TRef o = ones.t;
        o.dim = dd;
        o.str = dd.size() == 2 ? std::vector<int64_t>{mx, 1} : std::vector<int64_t>{1};
        o.lab = which;
        return o;
      };
      auto put = [&](int k, const TRef& src, const std::string& out_lab, const std::string& sum) {
        TRef dst = c->slot(0, I, J, k, out_lab);
        // the chi legs of the slot keep only the first (actual) indices
        TRef sub = dst;
        for (size_t q = 0; q < out_lab.size(); ++q) sub.dim[q] = src.dim[src.lab.find(out_lab[q])];
        contract(dev, c->st == T_F64 ? ctmk::MODE_F64 : ctmk::MODE_F32, sub, src, one(src, sum));
      };
      put(0, nb(-1, -1, "lurd"), "dr", "lu");
      put(1, nb(-1, 1, "lurd"), "ld", "ur");
      put(2, nb(1, 1, "lurd"), "ul", "rd");
      put(3, nb(1, -1, "lurd"), "ru", "ld");
      put(4, nb(-1, 0, "lurd"), "ldr", "u");
      put(5, nb(0, 1, "lurd"), "uld", "r");
      put(6, nb(1, 0, "lurd"), "rul", "d");
      put(7, nb(0, -1, "lurd"), "dru", "l");
    }
  c->have_prev = false;
}

// ---------------------------------------------------------------------------
// Half systems of the cut between rows I and I+1 at column step J of frame f
// (Fig. CTMRG c): N[(h w), (e z)] from the upper quadrants and S[(h v), (e x)]
// from the lower ones, written as float64 row-major matrices.
// Work queued between construction (with ``two``) and join() may go to the
// second stream; the main stream waits for it at join(), or when the scope is
// left early by an error.
struct SideScope {
  ctm_ctx* c;
  bool on;
  SideScope(ctm_ctx* cc, bool two) : c(cc), on(two) {
    if (on) c->fork();
  }
  void join() {
    if (!on) return;
    on = false;
    c->join();
  }
  ~SideScope() {
    if (!on) return;
    (void)hipEventRecord(c->ev_join, c->side.stream);
    (void)hipStreamWaitEvent(c->dev.stream, c->ev_join, 0);
  }
};

// out = X . s for the site s at frame-f position (I, J) with its legs
// (l, u, r, d) labelled ``lab``: the legs X shares with s are summed.  On the
// nested network s is the dense nested site.  On the double-layer network s
// is the reduced tensor a = sum_sigma A A* (legs of D^2, ket index major),
// and it is absorbed one layer at a time: the shared legs of X and the free
// legs of out are split into ket and bra halves, X is contracted with A over
// the ket halves, then with A* over sigma and the bra halves (Eq. Tred
// without forming a: 2 chi^2 D^6 d flops per quadrant instead of chi^2 D^8).
void absorb_site(ctm_ctx* c, Dev& dev, int m, const TRef& out, const TRef& X, int f, int I, int J,
                 const std::string& lab) {
  if (!c->layout) {
    contract(dev, m, out, X, c->site_t(f, I, J, lab));
    return;
  }
  const int64_t D = c->D, d = c->d, nk = d * D * D * D * D;
  std::string used = X.lab + out.lab + lab;
  auto fresh = [&]() {
    for (int ch = 33; ch < 127; ++ch)
      if (used.find((char)ch) == std::string::npos) {
        used += (char)ch;
        return (char)ch;
      }
    throw Error(CTM_EINVAL, "absorb_site: label pool exhausted");
  };
  const char sg = fresh();
  std::string kl, bl;
  TRef Xs = X, Os = out;
  for (char L : lab) {
    const char k = fresh(), b = fresh();
    kl += k;
    bl += b;
    if (Xs.lab.find(L) != std::string::npos) Xs = split_axis(Xs, L, D, D, k, b);
    else if (Os.lab.find(L) != std::string::npos) Os = split_axis(Os, L, D, D, k, b);
    else throw Error(CTM_EINVAL, "absorb_site: a site leg on neither side");
  }
  const int ii = ((I % c->ny(f)) + c->ny(f)) % c->ny(f), jj = ((J % c->nx(f)) + c->nx(f)) % c->nx(f);
  int oi, oj;
  c->to_orig(f, ii, jj, oi, oj);
  const int t = c->pattern[(size_t)oi * c->Lx + oj];
  void* Ap = (char*)c->a_frames.p + (size_t)(f * c->nt + t) * nk * type_size(c->st);
  TRef Ak = view(Ap, c->st, {d, D, D, D, D}, std::string(1, sg) + kl);
  TRef Ab = view(Ap, c->st, {d, D, D, D, D}, std::string(1, sg) + bl);
  // X . A over the ket halves of the shared legs
  std::string tl;
  std::vector<int64_t> td;
  for (size_t q = 0; q < Xs.lab.size(); ++q)
    if (kl.find(Xs.lab[q]) == std::string::npos) { tl += Xs.lab[q]; td.push_back(Xs.dim[q]); }
  for (size_t q = 0; q < Ak.lab.size(); ++q)
    if (Xs.lab.find(Ak.lab[q]) == std::string::npos) { tl += Ak.lab[q]; td.push_back(Ak.dim[q]); }
  Tmp T1(&dev, c->st, td, tl);
  contract(dev, m, T1.t, Xs, Ak);
  // then A* over sigma and the bra halves
  contract(dev, m, Os, T1.t, Ab);
}

void half_systems(ctm_ctx* c, Dev& dev, int f, int I, int J, double* Nout, double* Sout) {
  const int64_t chi = c->chi;
  const int m = c->mode;
  // upper-left quadrant: C1 T1 T4 s at (I, J)  ->  UL[c, r, e, z]
  TRef sUL = c->site_t(f, I, J, "yxrz");
  Tmp X1(&dev, c->st, {chi, sUL.dim[1], chi}, "axc");
  contract(dev, m, X1.t, c->slot(f, I, J, 0, "ab"), c->slot(f, I, J, 4, "bxc"));
  Tmp X2(&dev, c->st, {chi, sUL.dim[0], sUL.dim[1], chi}, "eyxc");
  contract(dev, m, X2.t, c->slot(f, I, J, 7, "eya"), X1.t);
  Tmp UL(&dev, c->st, {chi, sUL.dim[2], chi, sUL.dim[3]}, "crez");
  absorb_site(c, dev, m, UL.t, X2.t, f, I, J, "yxrz");
  // upper-right quadrant: T1 C2 T2 s at (I, J+1)  ->  UR[c, h, l, w]
  TRef sUR = c->site_t(f, I, J + 1, "lxyw");
  Tmp Y1(&dev, c->st, {chi, sUR.dim[1], chi}, "cxg");
  contract(dev, m, Y1.t, c->slot(f, I, J + 1, 4, "cxf"), c->slot(f, I, J + 1, 1, "fg"));
  Tmp Y2(&dev, c->st, {chi, sUR.dim[1], sUR.dim[2], chi}, "cxyh");
  contract(dev, m, Y2.t, Y1.t, c->slot(f, I, J + 1, 5, "gyh"));
  Tmp UR(&dev, c->st, {chi, chi, sUR.dim[0], sUR.dim[3]}, "chlw");
  absorb_site(c, dev, m, UR.t, Y2.t, f, I, J + 1, "lxyw");
  // lower-left quadrant: T4 C4 T3 s at (I+1, J)  ->  DL[c, e, x, r]
  TRef sDL = c->site_t(f, I + 1, J, "yxrw");
  Tmp Z1(&dev, c->st, {chi, sDL.dim[0], chi}, "bye");
  contract(dev, m, Z1.t, c->slot(f, I + 1, J, 3, "ba"), c->slot(f, I + 1, J, 7, "aye"));
  Tmp Z2(&dev, c->st, {chi, sDL.dim[3], sDL.dim[0], chi}, "cwye");
  contract(dev, m, Z2.t, c->slot(f, I + 1, J, 6, "cwb"), Z1.t);
  Tmp DL(&dev, c->st, {chi, chi, sDL.dim[1], sDL.dim[2]}, "cexr");
  absorb_site(c, dev, m, DL.t, Z2.t, f, I + 1, J, "yxrw");
  // lower-right quadrant: T2 C3 T3 s at (I+1, J+1)  ->  DR[h, c, l, v]
  TRef sDR = c->site_t(f, I + 1, J + 1, "lvyw");
  Tmp W1(&dev, c->st, {chi, sDR.dim[2], chi}, "hyf");
  contract(dev, m, W1.t, c->slot(f, I + 1, J + 1, 5, "hyg"), c->slot(f, I + 1, J + 1, 2, "gf"));
  Tmp W2(&dev, c->st, {chi, sDR.dim[2], sDR.dim[3], chi}, "hywc");
  contract(dev, m, W2.t, W1.t, c->slot(f, I + 1, J + 1, 6, "fwc"));
  Tmp DR(&dev, c->st, {chi, chi, sDR.dim[0], sDR.dim[1]}, "hclv");
  absorb_site(c, dev, m, DR.t, W2.t, f, I + 1, J + 1, "lvyw");

  const int64_t zdim = sUL.dim[3], wdim = sUR.dim[3], vdim = sDR.dim[1], xdim = sDL.dim[1];
  if (zdim != xdim || wdim != vdim) throw Error(CTM_EINVAL, "inconsistent nested bond dimensions");
  TRef Nv = view(Nout, T_F64, {chi, wdim, chi, zdim}, "hwez");
  TRef Sv = view(Sout, T_F64, {chi, vdim, chi, xdim}, "hvex");
  if (c->st == T_F64) {
    contract(dev, m, Nv, UR.t, relabel(UL.t, "clez"));
    contract(dev, m, Sv, DR.t, relabel(DL.t, "cexl"));
  } else {
    Tmp N32(&dev, c->st, {chi, wdim, chi, zdim}, "hwez");
    contract(dev, m, N32.t, UR.t, relabel(UL.t, "clez"));
    copy_into(dev, Nv, N32.t);
    Tmp S32(&dev, c->st, {chi, vdim, chi, xdim}, "hvex");
    contract(dev, m, S32.t, DR.t, relabel(DL.t, "cexl"));
    copy_into(dev, Sv, S32.t);
  }
}

// Batched Householder QR in place (qr_kernels.hip): matrix b is A + b*stride
// with element (i, j) at i*rs + j*cs; keeps tau and the T factor of every
// panel for applying Q later.
struct HQR {
  double* A = nullptr;
  int64_t m = 0, n = 0, k = 0, rs = 0, cs = 0, stride = 0;
  int batch = 0, nb = 16;
  int64_t npanel = 0;
  DBuf tau, T;
  int64_t tstride() const { return npanel * nb * nb; }
};

// Whether the panel kernel writes the dense V and Y of its block reflector
// itself (one launch less per panel); a process-wide switch, the results are
// identical.
bool g_qr_fused_vy = true;
// Whether a panel's trailing update runs as one launch
// (panel_update_mfma_kernel, the same arithmetic element for element) instead
// of the two matrix-core products with a split sum; a process-wide switch.
bool g_qr_one_update = true;

// C <- C - V (Y^T C) with the dense V, Y of panel p (L = m - j0 rows of nb per
// matrix): two FP64 MFMA products.
void hqr_panel_update(Dev& dev, const HQR& q, int64_t p, double* C, int64_t crs, int64_t ccs, int64_t cstride,
                      int64_t c0, int64_t ncols, void* V, void* Y) {
  const int64_t j0 = p * q.nb, L = q.m - j0;
  const int64_t nb = q.nb, B = q.batch;
  if (g_qr_one_update) {
    // the split over K that the contraction planner takes for Z = Y^T C (nb x
    // ncols outputs per matrix, K = L), so that the sums are the same
    const int64_t tiles = ((nb + 63) / 64) * ((ncols + 63) / 64) * B;
    int64_t kchunk = L, ksplit = 1;
    if (tiles < 128 && L >= 256) {
      const int64_t want = std::min<int64_t>((512 + tiles - 1) / tiles, L / 128);
      if (want > 1) {
        kchunk = ((L + want - 1) / want + 31) / 32 * 32;
        ksplit = (L + kchunk - 1) / kchunk;
      }
    }
    if (ksplit <= qrk::panel_update_max_split()) {
      // booked with the FP64 contractions it stands for (two products of 2 L nb ncols flops)
      g_counters.launches++;
      g_counters.flops += 4.0 * (double)L * nb * ncols * B;
      g_counters.count(ctmk::MODE_F64, 4.0 * (double)L * nb * ncols * B);
      if (g_counters.timing) g_counters.record(dev.stream, ctmk::MODE_F64);
      HIP_CHECK(qrk::launch_panel_update_mfma(C + j0 * crs + c0 * ccs, crs, ccs, cstride, L, ncols, q.nb,
                                              (const double*)V, (const double*)Y, q.batch, kchunk, (int)ksplit,
                                              dev.stream));
      if (g_counters.timing) g_counters.record(dev.stream, ctmk::MODE_F64);
      return;
    }
  }
  DBuf Z(&dev, (size_t)B * nb * ncols * 8);
  TRef Vv{V, T_F64, {B, L, nb}, {L * nb, nb, 1}, "brc"};
  TRef Yv{Y, T_F64, {B, L, nb}, {L * nb, nb, 1}, "brc"};
  TRef Cv{C + j0 * crs + c0 * ccs, T_F64, {B, L, ncols}, {cstride, crs, ccs}, "brn"};
  TRef Zv{Z.p, T_F64, {B, nb, ncols}, {nb * ncols, ncols, 1}, "bcn"};
  contract(dev, ctmk::MODE_F64, Zv, Yv, Cv);
  contract(dev, ctmk::MODE_F64, Cv, Vv, Zv, -1.0, 1);
}

// C_b[j0:m, c0:c0+ncols] <- H_p^T C_b (trans) or H_p C_b for the block
// reflector H_p = I - V T V^T of panel p: C <- C - V (Y^T C).
void hqr_panel_apply(Dev& dev, const HQR& q, int64_t p, double* C, int64_t crs, int64_t ccs, int64_t cstride,
                     int64_t c0, int64_t ncols, bool trans) {
  const int64_t j0 = p * q.nb, L = q.m - j0;
  const int nbp = (int)std::min<int64_t>(q.nb, q.k - j0);
  if (ncols <= 0 || L <= 0) return;
  const int64_t nb = q.nb, B = q.batch;
  DBuf V(&dev, (size_t)B * L * nb * 8), Y(&dev, (size_t)B * L * nb * 8);
  HIP_CHECK(qrk::launch_build_vy(q.A, q.rs, q.cs, q.stride, q.m, j0, nbp, q.nb, (const double*)q.T.p + p * nb * nb,
                                 q.tstride(), trans, (double*)V.p, (double*)Y.p, q.batch, dev.stream));
  hqr_panel_update(dev, q, p, C, crs, ccs, cstride, c0, ncols, V.p, Y.p);
}

void hqr_prepare(Dev& dev, HQR& q) {
  q.k = std::min(q.m, q.n);
  q.nb = qrk::panel_width(q.m);
  q.npanel = (q.k + q.nb - 1) / q.nb;
  q.tau = DBuf(&dev, (size_t)std::max<int64_t>(1, q.batch * q.k) * 8);
  q.T = DBuf(&dev, (size_t)std::max<int64_t>(1, q.batch * q.tstride()) * 8);
}

// Panel p of the blocked Householder QR and its update of the trailing columns.
void hqr_step(Dev& dev, HQR& q, int64_t p) {
  const int64_t j0 = p * q.nb;
  const int nbp = (int)std::min<int64_t>(q.nb, q.k - j0);
  double* Tp = (double*)q.T.p + p * q.nb * q.nb;
  const int64_t L = q.m - j0, ncols = q.n - (j0 + nbp);
  // the trailing update's V and Y, written by the panel kernel itself
  const bool fused = g_qr_fused_vy && ncols > 0 && L > 0;
  DBuf V, Y;
  if (fused) {
    V = DBuf(&dev, (size_t)q.batch * L * q.nb * 8);
    Y = DBuf(&dev, (size_t)q.batch * L * q.nb * 8);
  }
  if (g_counters.timing) g_counters.record(dev.stream, FAM_PANEL);
  HIP_CHECK(qrk::launch_panel(q.A, q.rs, q.cs, q.stride, q.m, q.n, j0, q.batch, (double*)q.tau.p, q.k, Tp,
                              q.tstride(), fused ? (double*)V.p : nullptr, fused ? (double*)Y.p : nullptr,
                              dev.stream));
  if (g_counters.timing) g_counters.record(dev.stream, FAM_PANEL);
  // Householder panel: about 4 (m - j0) nbp^2 flops per matrix (norms, reflections, T factor)
  g_counters.count(FAM_PANEL, 4.0 * (double)(q.m - j0) * nbp * nbp * q.batch);
  if (fused) hqr_panel_update(dev, q, p, q.A, q.rs, q.cs, q.stride, j0 + nbp, ncols, V.p, Y.p);
  else hqr_panel_apply(dev, q, p, q.A, q.rs, q.cs, q.stride, j0 + nbp, ncols, true);
}

void hqr_factor(Dev& dev, HQR& q) {
  hqr_prepare(dev, q);
  for (int64_t p = 0; p < q.npanel; ++p) hqr_step(dev, q, p);
}

// Factorisations on (possibly) different streams, their panels queued
// alternately: queued one after the other, the second stream would wait for
// the host to queue all of the first one's launches.
void hqr_factor_all(Dev* const* devs, HQR* const* qs, int count) {
  int64_t most = 0;
  for (int i = 0; i < count; ++i) {
    hqr_prepare(*devs[i], *qs[i]);
    most = std::max(most, qs[i]->npanel);
  }
  for (int64_t p = 0; p < most; ++p)
    for (int i = 0; i < count; ++i)
      if (p < qs[i]->npanel) hqr_step(*devs[i], *qs[i], p);
}

// C_b <- Q_b C_b (trans: Q_b^T C_b) for the m x ncols matrices C + b*cstride
// with element (i, j) at i*crs + j*ccs.
void hqr_apply(Dev& dev, const HQR& q, double* C, int64_t crs, int64_t ccs, int64_t cstride, int64_t ncols, bool trans) {
  for (int64_t t = 0; t < q.npanel; ++t) {
    const int64_t p = trans ? t : q.npanel - 1 - t;
    hqr_panel_apply(dev, q, p, C, crs, ccs, cstride, 0, ncols, trans);
  }
}

// SVD of the r x r column-major matrices A[b] (stride r*r) by one-sided
// Jacobi with QR preconditioning: A = Q R (Householder), the columns of
// X = R^T are rotated until mutually orthogonal, X W = U_X diag(s), so that
// A = (Q W) diag(s) U_X^T.  Starting from R^T instead of A cuts the number of
// Jacobi sweeps about threefold on the graded spectra of CTMRG.  The sweeps
// are blocked: each round of a tournament over blocks of columns rotates every
// block pair in one workgroup.  When the device holds the whole grid, one
// launch runs all rounds and sweeps and takes the stop test itself
// (bjac_svd_kernel), so the host does not wait for the SVD; otherwise each
// round is a launch (bjac_round_kernel) and the host tests after each sweep.
// Both run the same rounds and give identical results.  Outputs: all
// r singular values, descending, to sv[b]; the kmax leading left vectors to
// U[b] and right vectors to Vk[b] (column-major r x kmax).  A is overwritten.
int jacobi_svd(ctm_ctx* c, double* A, int64_t r, int batch, int64_t kmax, double* sv, double* U, double* Vk) {
  Dev& dev = c->dev;
  const int64_t stride = r * r;
  const int maxsw = c->jacobi_max_sweeps;
  // the whole iteration in one launch when the device holds all its workgroups at once
  if (c->sweep_capacity < 0) c->sweep_capacity = ctmk::bjac_sweep_capacity();
  // a cooperative launch is refused by the runtime when the device cannot hold
  // the grid; the plain launch is only taken when the occupancy says it can
  bool one_launch = c->jacobi_one_launch && (c->jacobi_coop || ctmk::bjac_grid(r, batch) <= c->sweep_capacity);
  // per-sweep rotation counts and largest rotated |cos| (one slot per sweep in
  // one launch, one reused slot otherwise), then the sweep count; the
  // synchronisation words of the one-launch iteration
  const int64_t slots = one_launch ? (int64_t)maxsw * batch : batch;
  const int64_t nsync = one_launch ? ctmk::bjac_sync_words(r, batch, maxsw) : 0;
  DBuf X(&dev, (size_t)batch * stride * 8), W(&dev, (size_t)batch * stride * 8),
      rot(&dev, (size_t)(slots + 1 + nsync) * sizeof(int)), tiny2(&dev, (size_t)batch * 8),
      ovl(&dev, (size_t)slots * 8);
  HQR qm;
  qm.A = A; qm.m = r; qm.n = r; qm.rs = 1; qm.cs = r; qm.stride = stride; qm.batch = batch;
  hqr_factor(dev, qm);
  HIP_CHECK(ctmk::launch_rt_from_qr(A, (double*)X.p, r, stride, batch, dev.stream));
  HIP_CHECK(ctmk::launch_identity((double*)W.p, r, stride, batch, dev.stream));
  DBuf fwork(&dev, (size_t)std::max(ctmk::frob_tiny_work_doubles(batch), ctmk::jacobi_finish_work_doubles(r, batch)) * 8);
  HIP_CHECK(ctmk::launch_frob_tiny((const double*)X.p, stride, stride, batch, 2.2e-16, (double*)tiny2.p,
                                   (double*)fwork.p, dev.stream));
  const double tol = std::max(1e-15, 2.2e-16 * std::sqrt((double)r));
  // The method converges quadratically at the end: once the largest |cos| of
  // a pair rotated in a whole sweep is at most sqrt(tol), what that sweep left
  // is of order tol, which is what a further sweep (rotations at the rounding
  // level) and the final sweep without rotations would certify.
  const double stop = std::sqrt(tol);
  const int64_t rounds = ctmk::bjac_rounds(r);
  // algorithmic flops of one round: per block pair of C columns of length r, the
  // Gram matrix (C(C+1)/2 dot products) and the rotation of the pair's columns
  // of X and W (two r x C by C x C products); the inner Jacobi on C x C is not counted
  const double Cw = (double)ctmk::bjac_pair_columns();
  const double pairs = (double)(ctmk::bjac_rounds(r) + 1) / 2.0 * batch;
  const double bj_flops = pairs * ((Cw * (Cw + 1) / 2.0) * 2.0 * r + 2.0 * (2.0 * r * Cw * Cw));
  int* rot_p = (int*)rot.p;
  int sweep = 0;
  if (one_launch) {
    // no host synchronisation: failures reach the context's solver flag,
    // which the calls check when they return
    HIP_CHECK(ctmk::launch_fill_int(rot_p, 0, slots + 1 + nsync, dev.stream));
    fill(dev, view(ovl.p, T_F64, {slots}, "b"), 0.0);
    if (g_counters.timing) g_counters.record(dev.stream, FAM_JACOBI);
    hipError_t e = ctmk::launch_bjac_svd((double*)X.p, (double*)W.p, r, stride, batch, maxsw, tol, stop,
                                         (const double*)tiny2.p, rot_p, (double*)ovl.p, (unsigned*)(rot_p + slots + 1),
                                         (int*)c->flag.p + 1, rot_p + slots, c->jacobi_coop, dev.stream);
    if (e != hipSuccess && c->jacobi_coop) {
      // refused (the grid does not fit the device at once): nothing was queued;
      // clear the error, close the timed interval (empty) and take one launch
      // per round below
      (void)hipGetLastError();
      if (g_counters.timing) g_counters.record(dev.stream, FAM_JACOBI);
      one_launch = false;
    } else {
      HIP_CHECK(e);
    }
  }
  if (one_launch) {
    if (g_counters.timing) {
      g_counters.record(dev.stream, FAM_JACOBI);
      // profiling only: the flop count needs the number of sweeps run
      HIP_CHECK(hipMemcpyAsync(&sweep, rot_p + slots, sizeof(int), hipMemcpyDeviceToHost, dev.stream));
      HIP_CHECK(hipStreamSynchronize(dev.stream));
      g_counters.count(FAM_JACOBI, bj_flops * (double)rounds * sweep);
    }
  } else {
    std::vector<int> h(batch);
    std::vector<double> ho(batch);
    for (sweep = 1; sweep <= maxsw; ++sweep) {
      HIP_CHECK(ctmk::launch_fill_int(rot_p, 0, batch, dev.stream));
      fill(dev, view(ovl.p, T_F64, {(int64_t)batch}, "b"), 0.0);
      for (int64_t t = 0; t < rounds; ++t) {
        if (g_counters.timing) g_counters.record(dev.stream, FAM_JACOBI);
        HIP_CHECK(ctmk::launch_bjac_round((double*)X.p, (double*)W.p, r, stride, batch, (int)t, tol,
                                          (const double*)tiny2.p, 1, rot_p, (double*)ovl.p, dev.stream));
        if (g_counters.timing) g_counters.record(dev.stream, FAM_JACOBI);
        g_counters.count(FAM_JACOBI, bj_flops);
      }
      HIP_CHECK(hipMemcpyAsync(h.data(), rot_p, batch * sizeof(int), hipMemcpyDeviceToHost, dev.stream));
      HIP_CHECK(hipMemcpyAsync(ho.data(), ovl.p, batch * sizeof(double), hipMemcpyDeviceToHost, dev.stream));
      HIP_CHECK(hipStreamSynchronize(dev.stream));
      bool any = false;
      double big = 0.0;
      for (int b = 0; b < batch; ++b) {
        any |= h[b] != 0;
        big = std::max(big, ho[b]);
      }
      if (!any || big <= stop) break;
    }
    if (sweep > maxsw) throw Error(CTM_ESOLVER, "Jacobi SVD did not converge");
  }
  // normalised columns of X W are the right vectors of A; the columns of W, times Q, the left ones
  HIP_CHECK(ctmk::launch_jacobi_finish((const double*)X.p, (const double*)W.p, r, stride, batch, kmax, sv, Vk, U,
                                       (double*)fwork.p, dev.stream));
  hqr_apply(dev, qm, U, 1, r, r * kmax, kmax, false);
  return sweep;
}

// Leading singular triplets of the r x r column-major matrices M[b] (stride
// r*r) from a randomized range finder (Halko, Martinsson and Tropp, SIAM Rev.
// 53 (2011), Algorithms 4.4 and 5.1), the cheaper projectors of the paper's
// outlook: k = min(chi + oversample, r) columns, the test matrix Omega[i][j] =
// 2u - 1 with u = (splitmix64(seed, i k + j) >> 11) 2^-53, Y = M Omega and
// ``power`` passes of Z = M^T Q, Y = M Q(Z), every product orthonormalised by
// the blocked Householder QR; then B^T = M^T Q = Q_b R_b, the SVD R_b^T =
// U_r diag(s) V_r^T of the k x k factor by the block Jacobi, and M ~ (Q U_r)
// diag(s) (Q_b V_r)^T.  Outputs as jacobi_svd: s (k values, then zeros, to the
// r slots of sv[b]), the kmax leading left and right vectors to U[b], Vk[b]
// (column-major r x kmax, columns beyond k zero).  M is left unchanged.
void randomized_svd(ctm_ctx* c, const double* M, int64_t r, int batch, int64_t kmax, double* sv, double* U, double* Vk) {
  Dev& dev = c->dev;
  const int m = ctmk::MODE_F64;
  const int64_t k = std::min<int64_t>(c->chi + c->rsvd_oversample, r);
  const int64_t rk = r * k;
  DBuf Om(&dev, (size_t)rk * 8), Q(&dev, (size_t)batch * rk * 8), Z(&dev, (size_t)batch * rk * 8),
      ones(&dev, (size_t)batch * k * 8);
  HIP_CHECK(optk::launch_uniform_init_f64((double*)Om.p, rk, c->rsvd_seed, 0, 1.0, dev.stream));
  fill(dev, view(ones.p, T_F64, {batch * k}, "q"), 1.0);
  TRef Mv{(void*)M, T_F64, {batch, r, r}, {r * r, 1, r}, "bij"};
  auto colmaj = [&](void* p, const std::string& lab) { return TRef{p, T_F64, {batch, r, k}, {rk, 1, r}, lab}; };
  // Y (in place) -> the explicit thin Q factor of its Householder QR, written to ``out``
  auto orth = [&](DBuf& Y, DBuf& out) {
    HQR q;
    q.A = (double*)Y.p; q.m = r; q.n = k; q.rs = 1; q.cs = r; q.stride = rk; q.batch = batch;
    hqr_factor(dev, q);
    fill(dev, view(out.p, T_F64, {batch * rk}, "q"), 0.0);
    copy_into(dev, TRef{out.p, T_F64, {batch, k}, {rk, r + 1}, "bd"}, view(ones.p, T_F64, {batch, k}, "bd"));
    hqr_apply(dev, q, (double*)out.p, 1, r, rk, k, false);
  };
  DBuf Y(&dev, (size_t)batch * rk * 8);
  contract(dev, m, colmaj(Y.p, "bil"), Mv, view(Om.p, T_F64, {r, k}, "jl"));
  orth(Y, Q);
  for (int p = 0; p < c->rsvd_power; ++p) {
    contract(dev, m, colmaj(Z.p, "bjl"), Mv, colmaj(Q.p, "bil"));
    orth(Z, Y);   // Y holds Q(Z)
    contract(dev, m, colmaj(Z.p, "bil"), Mv, colmaj(Y.p, "bjl"));
    orth(Z, Q);
  }
  // B^T = M^T Q = Q_b R_b; the Jacobi SVD of the k x k factor R_b^T
  contract(dev, m, colmaj(Z.p, "bjl"), Mv, colmaj(Q.p, "bil"));
  HQR qb;
  qb.A = (double*)Z.p; qb.m = r; qb.n = k; qb.rs = 1; qb.cs = r; qb.stride = rk; qb.batch = batch;
  hqr_factor(dev, qb);
  const int64_t km = std::min(kmax, k);
  DBuf L(&dev, (size_t)batch * k * k * 8), ss(&dev, (size_t)batch * k * 8), Ur(&dev, (size_t)batch * k * km * 8),
      Vr(&dev, (size_t)batch * k * km * 8);
  HIP_CHECK(qrk::launch_extract_rt((const double*)Z.p, 1, r, rk, k, k, (double*)L.p, k * k, batch, dev.stream));
  jacobi_svd(c, (double*)L.p, k, batch, km, (double*)ss.p, (double*)Ur.p, (double*)Vr.p);
  // singular values into the r slots of every matrix (zeros beyond k)
  fill(dev, view(sv, T_F64, {batch * r}, "q"), 0.0);
  copy_into(dev, TRef{sv, T_F64, {batch, k}, {r, 1}, "bq"}, view(ss.p, T_F64, {batch, k}, "bq"));
  // U = Q U_r, V = Q_b [V_r; 0]
  fill(dev, view(U, T_F64, {batch * r * kmax}, "q"), 0.0);
  fill(dev, view(Vk, T_F64, {batch * r * kmax}, "q"), 0.0);
  contract(dev, m, TRef{U, T_F64, {batch, r, km}, {r * kmax, 1, r}, "bia"}, colmaj(Q.p, "bil"),
           TRef{Ur.p, T_F64, {batch, k, km}, {k * km, 1, k}, "bla"});
  copy_into(dev, TRef{Vk, T_F64, {batch, k, km}, {r * kmax, 1, r}, "bla"},
            TRef{Vr.p, T_F64, {batch, k, km}, {k * km, 1, k}, "bla"});
  hqr_apply(dev, qb, Vk, 1, r, r * kmax, km, false);
}

// Projectors of every row of column step J of frame f (Eqs. PQ, QRSVD), in
// float64, written to P64/Q64 + I*maxkd*chi as [(chi-leg, site-leg), chi]
// matrices (the site leg is the down leg of (I, J)).
//
// Rows of equal parity have equal shapes and are handled together.  N and S
// are mn x kd (rows: right cut, columns: left cut a5a6), stored row-major and
// factorised in place by the batched Householder QR (N = Q_n R_n, R_n r x kd,
// r = min(kd, mn) = chi*D, Eq. QRSVD); L = R^T is kept column-major
// (kd x r); then M = R_n R_s^T = L_n^T L_s,
// M = U diag(s) V^T, P = R_s^T V w = L_s V w and Q = R_n^T U w = L_n U w with
// w_k = s_k^(-1/2) for the chi largest s_k above cutoff * s_1 (zero
// otherwise).  The QR is taken also when N is not tall: forming N S^T
// directly loses the accuracy of the small kept singular values that the
// triangular factors preserve.
//
// While the tape records, all r singular triplets are kept together with the
// singular vectors of rho = N S^T (U_rho = Q_n [U; 0], V_rho = Q_s [V; 0])
// and the derivative of the block (N, S) -> (P, Q) is recorded (see
// proj_backward).
// Largest singular value of M, relative to |N|_F |S|_F, at or below which a
// cut carries no weight (rounding alone leaves about 1e-16).
constexpr double kEmptyCut = 1e-12;

void proj_backward(ctm_ctx* c, const ProjRow& R, int64_t r);

void column_projectors(ctm_ctx* c, int f, int J, double* P64, double* Q64, int64_t maxkd) {
  Dev& dev = c->dev;
  const int a = c->ny(f);
  const int64_t chi = c->chi;
  const int m = c->mode;
  const bool rec = c->tape.recording();
  int64_t kd[2] = {0, 0}, mn[2] = {0, 0};
  int cnt[2] = {0, 0};
  for (int I = 0; I < a; ++I) {
    int p = I & 1;
    kd[p] = chi * c->site(f, I, J).dim[3];
    mn[p] = chi * c->site(f, I, J + 1).dim[3];
    cnt[p]++;
  }
  const int64_t r = std::min(kd[0], mn[0]);
  for (int p = 0; p < 2; ++p)
    if (cnt[p] && std::min(kd[p], mn[p]) != r) throw Error(CTM_EINVAL, "rows of a column step differ in rank bound");
  // per parity: N of the rows at 0..cnt-1, S at cnt..2cnt-1 (row-major mn x kd each)
  DBuf NS[2];
  for (int p = 0; p < 2; ++p)
    if (cnt[p]) NS[p] = DBuf(&dev, (size_t)2 * cnt[p] * kd[p] * mn[p] * 8);
  auto Nptr = [&](int p, int b) { return (double*)NS[p].p + (size_t)b * kd[p] * mn[p]; };
  auto Sptr = [&](int p, int b) { return (double*)NS[p].p + (size_t)(cnt[p] + b) * kd[p] * mn[p]; };
  // a recomputed sweep takes its projector block from the forward pass
  // (recorded, so one device stream); a forward sweep that will be
  // recomputed keeps all r triplets and U_rho, V_rho as a recorded one does
  std::vector<ProjCacheStep>* use = rec ? c->pc_use : nullptr;
  std::vector<ProjCacheStep>* keep = rec ? nullptr : c->pc_fill;
  const int64_t kk = (rec || keep) ? r : chi;   // singular vectors kept per row
  HQR qr[2];
  DBuf L[2];   // R^T of N (first cnt) and S (next cnt): column-major kd x r
  DBuf Mb, sv, Uk, Vk, w;
  if (!use) {
    TapePause hold(dev);   // workspaces of the projector block, not recorded buffers
    Mb = DBuf(&dev, (size_t)a * r * r * 8);
    sv = DBuf(&dev, (size_t)a * r * 8);
    Uk = DBuf(&dev, (size_t)a * r * kk * 8);
    Vk = DBuf(&dev, (size_t)a * r * kk * 8);
    w = DBuf(&dev, (size_t)a * chi * 8);
    for (int p = 0; p < 2; ++p)
      if (cnt[p]) L[p] = DBuf(&dev, (size_t)2 * cnt[p] * kd[p] * r * 8);
  }
  // not recorded and both parities present: the odd rows (half systems, QR,
  // their part of M) run on the second stream; the results are identical.
  // Every block of the main stream's cache that the second stream writes (NS,
  // L, Mb) is taken before the fork: a block freed after it may still be in
  // use by main-stream kernels queued after the fork.
  const bool two = !rec && c->streams > 1 && cnt[0] && cnt[1];
  Dev& pdev1 = two ? c->side : dev;
  SideScope side_scope(c, two);
  for (int I = 0; I < a; ++I) {
    int p = I & 1, b = I >> 1;
    half_systems(c, p ? pdev1 : dev, f, I, J, Nptr(p, b), Sptr(p, b));
  }
  TapePause pause(dev);   // the block below is one recorded operation
  std::vector<ProjRow> rows((rec || keep) ? a : 0);
  if (rec)
    for (int I = 0; I < a; ++I) {
      int p = I & 1, b = I >> 1;
      ProjRow& R = rows[I];
      R.kd = kd[p]; R.mn = mn[p];
      const size_t sz = (size_t)kd[p] * mn[p];
      R.Nadj = Nptr(p, b);
      R.Sadj = Sptr(p, b);
      R.N = std::make_shared<DBuf>(&dev, sz * 8);
      R.S = std::make_shared<DBuf>(&dev, sz * 8);
      HIP_CHECK(hipMemcpyAsync(R.N->p, R.Nadj, sz * 8, hipMemcpyDeviceToDevice, dev.stream));
      HIP_CHECK(hipMemcpyAsync(R.S->p, R.Sadj, sz * 8, hipMemcpyDeviceToDevice, dev.stream));
      R.P = P64 + (size_t)I * maxkd * chi;
      R.Q = Q64 + (size_t)I * maxkd * chi;
    }
  if (use) {
    if (c->pc_pos >= use->size()) throw Error(CTM_EINVAL, "projector cache: recomputed sweep out of step");
    const ProjCacheStep& st = (*use)[c->pc_pos++];
    if (st.rows != a || st.maxkd != maxkd) throw Error(CTM_EINVAL, "projector cache: recomputed sweep out of step");
    const size_t pb = (size_t)a * maxkd * chi * 8;
    HIP_CHECK(hipMemcpyAsync(P64, st.P.p, pb, hipMemcpyDeviceToDevice, dev.stream));
    HIP_CHECK(hipMemcpyAsync(Q64, st.Q.p, pb, hipMemcpyDeviceToDevice, dev.stream));
    for (int I = 0; I < a; ++I) {
      rows[I].Ur = st.saved[I].Ur;
      rows[I].Vr = st.saved[I].Vr;
      rows[I].s = st.saved[I].s;
      rows[I].w = st.saved[I].w;
    }
    c->tape.custom([c, rows, r]() {
      for (const ProjRow& R : rows) proj_backward(c, R, r);
    });
    return;
  }
  {
    Dev* fdev[2];
    HQR* fq[2];
    int nf = 0;
    for (int p = 0; p < 2; ++p) {
      if (!cnt[p]) continue;
      const int64_t sz = kd[p] * mn[p];
      qr[p].A = (double*)NS[p].p;
      qr[p].m = mn[p]; qr[p].n = kd[p]; qr[p].rs = kd[p]; qr[p].cs = 1; qr[p].stride = sz; qr[p].batch = 2 * cnt[p];
      fdev[nf] = p ? &pdev1 : &dev;
      fq[nf++] = &qr[p];
    }
    hqr_factor_all(fdev, fq, nf);
  }
  for (int p = 0; p < 2; ++p) {
    if (!cnt[p]) continue;
    Dev& pd = p ? pdev1 : dev;
    const int64_t sz = kd[p] * mn[p];
    HIP_CHECK(qrk::launch_extract_rt((const double*)NS[p].p, kd[p], 1, sz, kd[p], r, (double*)L[p].p, kd[p] * r,
                                     2 * cnt[p], pd.stream));
    TRef Mv{(double*)Mb.p + (size_t)p * r * r, T_F64, {cnt[p], r, r}, {2 * r * r, 1, r}, "bij"};
    TRef Lnv{L[p].p, T_F64, {cnt[p], kd[p], r}, {kd[p] * r, 1, kd[p]}, "bai"};
    TRef Lsv{(double*)L[p].p + (size_t)cnt[p] * kd[p] * r, T_F64, {cnt[p], kd[p], r}, {kd[p] * r, 1, kd[p]}, "baj"};
    contract(pd, m, Mv, Lnv, Lsv);
  }
  side_scope.join();
  // rows are interleaved by parity in Mb: row I at I*r*r (p + 2b)
  if (!rec && !keep && c->svd_method == 1)
    randomized_svd(c, (const double*)Mb.p, r, a, kk, (double*)sv.p, (double*)Uk.p, (double*)Vk.p);
  else jacobi_svd(c, (double*)Mb.p, r, a, kk, (double*)sv.p, (double*)Uk.p, (double*)Vk.p);
  {
    // a cut whose bond density matrix vanishes to working precision has no
    // projector (Lambda~^(-1/2) of Eq. PQ is undefined): counted in the flags
    // and reported as CTM_ESOLVER when the call returns
    ctmk::CutList cl;
    std::memset(&cl, 0, sizeof(cl));
    for (int I = 0; I < a; ++I) {
      int p = I & 1, b = I >> 1;
      const size_t lfs = (size_t)kd[p] * r;
      cl.Ln[I] = (const double*)L[p].p + (size_t)b * lfs;
      cl.Ls[I] = (const double*)L[p].p + (size_t)(cnt[p] + b) * lfs;
      cl.s1[I] = (const double*)sv.p + (size_t)I * r;
      cl.n[I] = (int64_t)lfs;
    }
    DBuf cw(&dev, (size_t)a * ctmk::CUT_CHUNKS * 2 * 8);
    HIP_CHECK(ctmk::launch_cut_check(cl, a, kEmptyCut, (double*)cw.p, (int*)c->flag.p + 2, dev.stream));
  }
  HIP_CHECK(ctmk::launch_svd_weights((const double*)sv.p, r, r, (double*)w.p, chi, c->cutoff, a, dev.stream));
  for (int I = 0; I < a; ++I) {
    int p = I & 1, b = I >> 1;
    const int64_t lfs = kd[p] * r;
    TRef Lv{(void*)((double*)L[p].p + (size_t)b * lfs), T_F64, {kd[p], r}, {1, kd[p]}, "ai"};
    TRef Rv{(void*)((double*)L[p].p + (size_t)(cnt[p] + b) * lfs), T_F64, {kd[p], r}, {1, kd[p]}, "ai"};
    TRef Uv{(double*)Uk.p + (size_t)I * r * kk, T_F64, {r, chi}, {1, r}, "ik"};
    TRef Vv{(double*)Vk.p + (size_t)I * r * kk, T_F64, {r, chi}, {1, r}, "ik"};
    const double* wI = (const double*)w.p + (size_t)I * chi;
    contract(dev, m, view(P64 + (size_t)I * maxkd * chi, T_F64, {kd[p], chi}, "ak"), Rv, Vv, 1.0, 0, wI);
    contract(dev, m, view(Q64 + (size_t)I * maxkd * chi, T_F64, {kd[p], chi}, "ak"), Lv, Uv, 1.0, 0, wI);
  }
  {
    // gauge: each kept pair (u_k, v_k) takes the sign that makes the first
    // entry of P[:, k] within a relative 1e-9 of its largest magnitude
    // positive; P does not depend on the QR's
    // sign conventions, so the converged environment is a fixed point of the
    // sweep entry by entry
    ctmk::SignList sl;
    std::memset(&sl, 0, sizeof(sl));
    for (int I = 0; I < a; ++I) {
      sl.P[I] = P64 + (size_t)I * maxkd * chi;
      sl.Q[I] = Q64 + (size_t)I * maxkd * chi;
      sl.U[I] = (double*)Uk.p + (size_t)I * r * kk;
      sl.V[I] = (double*)Vk.p + (size_t)I * r * kk;
      sl.kd[I] = kd[I & 1];
    }
    HIP_CHECK(ctmk::launch_proj_signs(sl, a, std::min<int64_t>(chi, r), r, dev.stream));
  }
  if (!rec && !keep) return;
  // singular vectors of rho = N S^T: U_rho = Q_n [U; 0], V_rho = Q_s [V; 0]
  for (int p = 0; p < 2; ++p) {
    if (!cnt[p]) continue;
    const int64_t mnp = mn[p];
    DBuf C(&dev, (size_t)2 * cnt[p] * mnp * r * 8);   // column-major mn x r, N rows then S rows
    fill(dev, view(C.p, T_F64, {2 * cnt[p] * mnp * r}, "q"), 0.0);
    for (int side = 0; side < 2; ++side)
      for (int b = 0; b < cnt[p]; ++b) {
        const int I = 2 * b + p;
        const double* src = (double*)(side == 0 ? Uk : Vk).p + (size_t)I * r * kk;
        double* dst = (double*)C.p + (size_t)(side * cnt[p] + b) * mnp * r;
        copy_into(dev, TRef{dst, T_F64, {r, r}, {1, mnp}, "ij"}, TRef{(void*)src, T_F64, {r, r}, {1, r}, "ij"});
      }
    hqr_apply(dev, qr[p], (double*)C.p, 1, mnp, mnp * r, r, false);
    for (int b = 0; b < cnt[p]; ++b) {
      ProjRow& R = rows[2 * b + p];
      R.Ur = std::make_shared<DBuf>(&dev, (size_t)mnp * r * 8);
      R.Vr = std::make_shared<DBuf>(&dev, (size_t)mnp * r * 8);
      HIP_CHECK(hipMemcpyAsync(R.Ur->p, (double*)C.p + (size_t)b * mnp * r, (size_t)mnp * r * 8,
                               hipMemcpyDeviceToDevice, dev.stream));
      HIP_CHECK(hipMemcpyAsync(R.Vr->p, (double*)C.p + (size_t)(cnt[p] + b) * mnp * r, (size_t)mnp * r * 8,
                               hipMemcpyDeviceToDevice, dev.stream));
    }
  }
  for (int I = 0; I < a; ++I) {
    ProjRow& R = rows[I];
    R.s = std::make_shared<DBuf>(&dev, (size_t)r * 8);
    R.w = std::make_shared<DBuf>(&dev, (size_t)chi * 8);
    HIP_CHECK(hipMemcpyAsync(R.s->p, (double*)sv.p + (size_t)I * r, r * 8, hipMemcpyDeviceToDevice, dev.stream));
    HIP_CHECK(hipMemcpyAsync(R.w->p, (double*)w.p + (size_t)I * chi, chi * 8, hipMemcpyDeviceToDevice, dev.stream));
  }
  if (keep) {
    keep->emplace_back();
    ProjCacheStep& st = keep->back();
    st.rows = a;
    st.maxkd = maxkd;
    const size_t pb = (size_t)a * maxkd * chi * 8;
    st.P = DBuf(&dev, pb);
    st.Q = DBuf(&dev, pb);
    HIP_CHECK(hipMemcpyAsync(st.P.p, P64, pb, hipMemcpyDeviceToDevice, dev.stream));
    HIP_CHECK(hipMemcpyAsync(st.Q.p, Q64, pb, hipMemcpyDeviceToDevice, dev.stream));
    st.saved = std::move(rows);
    return;
  }
  c->tape.custom([c, rows, r]() {
    for (const ProjRow& R : rows) proj_backward(c, R, r);
  });
}

// Adjoint of (N, S) -> (P, Q) for one row, in the form P = S^T V_rho w,
// Q = N^T U_rho w with rho = N S^T = U_rho diag(s) V_rho^T (thin, all r
// triplets), which needs no inverse of the triangular factors:
//   Sbar += X Pbar^T, Nbar += Y Qbar^T with X = V_rho[:, :chi] w, Y = U_rho[:, :chi] w;
//   Ubar = (N Qbar) w, Vbar = (S Pbar) w on the first chi columns;
//   sbar_k = -1/2 w_k^3 (<V_rho_k, S Pbar_k> + <U_rho_k, N Qbar_k>);
//   rhobar from the thin-SVD derivative with the Lorentzian-broadened F
//   (Eq. AD; F_ij = D/(D^2 + (eta max(s_i^2, s_j^2))^2), D = s_j^2 - s_i^2);
//   Nbar += rhobar S, Sbar += rhobar^T N.
void proj_backward(ctm_ctx* c, const ProjRow& R, int64_t r) {
  Dev& dev = c->dev;
  Tape& tp = c->tape;
  const int64_t chi = c->chi, kd = R.kd, mn = R.mn;
  const int m = ctmk::MODE_F64;
  double* Nc = (double*)R.N->p;
  double* Sc = (double*)R.S->p;
  double* Ur = (double*)R.Ur->p;
  double* Vr = (double*)R.Vr->p;
  const double* sv = (const double*)R.s->p;
  const double* w = (const double*)R.w->p;
  TRef Pb = view(tp.adj_ptr(R.P), T_F64, {kd, chi}, "ak");
  TRef Qb = view(tp.adj_ptr(R.Q), T_F64, {kd, chi}, "ak");
  TRef Nb = view(tp.adj_ptr(R.Nadj), T_F64, {mn, kd}, "ia");
  TRef Sb = view(tp.adj_ptr(R.Sadj), T_F64, {mn, kd}, "ia");
  TRef Nv = view(Nc, T_F64, {mn, kd}, "ia"), Sv = view(Sc, T_F64, {mn, kd}, "ia");
  TRef Urv{Ur, T_F64, {mn, r}, {1, mn}, "iq"}, Vrv{Vr, T_F64, {mn, r}, {1, mn}, "iq"};
  DBuf X(&dev, (size_t)mn * chi * 8), Y(&dev, (size_t)mn * chi * 8), Xb(&dev, (size_t)mn * chi * 8),
      Yb(&dev, (size_t)mn * chi * 8);
  HIP_CHECK(ctmk::launch_colscale_copy(Vr, 1, mn, mn, chi, w, (double*)X.p, dev.stream));
  HIP_CHECK(ctmk::launch_colscale_copy(Ur, 1, mn, mn, chi, w, (double*)Y.p, dev.stream));
  contract(dev, m, Sb, view(X.p, T_F64, {mn, chi}, "ik"), Pb, 1.0, 1);
  contract(dev, m, Nb, view(Y.p, T_F64, {mn, chi}, "ik"), Qb, 1.0, 1);
  contract(dev, m, view(Xb.p, T_F64, {mn, chi}, "ik"), Sv, Pb);
  contract(dev, m, view(Yb.p, T_F64, {mn, chi}, "ik"), Nv, Qb);
  DBuf sb(&dev, (size_t)r * 8);
  HIP_CHECK(ctmk::launch_svd_sbar(Ur, Vr, (const double*)Xb.p, (const double*)Yb.p, mn, r, chi, w, (double*)sb.p,
                                  dev.stream));
  // Ubar = Yb w, Vbar = Xb w (first chi columns)
  DBuf Ubar(&dev, (size_t)mn * chi * 8), Vbar(&dev, (size_t)mn * chi * 8);
  HIP_CHECK(ctmk::launch_colscale_copy((const double*)Yb.p, chi, 1, mn, chi, w, (double*)Ubar.p, dev.stream));
  HIP_CHECK(ctmk::launch_colscale_copy((const double*)Xb.p, chi, 1, mn, chi, w, (double*)Vbar.p, dev.stream));
  TRef Ubv = view(Ubar.p, T_F64, {mn, chi}, "ik"), Vbv = view(Vbar.p, T_F64, {mn, chi}, "ik");
  DBuf G(&dev, (size_t)r * chi * 8), Hm(&dev, (size_t)r * chi * 8);
  contract(dev, m, view(G.p, T_F64, {r, chi}, "qk"), Urv, Ubv);
  contract(dev, m, view(Hm.p, T_F64, {r, chi}, "qk"), Vrv, Vbv);
  DBuf core(&dev, (size_t)r * r * 8);
  HIP_CHECK(ctmk::launch_svd_core((const double*)G.p, (const double*)Hm.p, sv, (const double*)sb.p, r, chi, c->eta,
                                  (double*)core.p, dev.stream));
  // Gm = Ur core + [ (Ubar - Ur G) sinv , 0 ]
  DBuf Gm(&dev, (size_t)mn * r * 8), T(&dev, (size_t)mn * chi * 8), A2(&dev, (size_t)mn * chi * 8);
  TRef Gmv = view(Gm.p, T_F64, {mn, r}, "ip");
  contract(dev, m, Gmv, Urv, view(core.p, T_F64, {r, r}, "qp"));
  contract(dev, m, view(T.p, T_F64, {mn, chi}, "ik"), Urv, view(G.p, T_F64, {r, chi}, "qk"));
  HIP_CHECK(ctmk::launch_sub_sinv((const double*)Ubar.p, (const double*)T.p, mn, chi, sv, w, (double*)A2.p, dev.stream));
  TRef Gm_k{Gm.p, T_F64, {mn, chi}, {r, 1}, "ik"};
  copy_into(dev, Gm_k, view(A2.p, T_F64, {mn, chi}, "ik"), true);
  // B2 = (Vbar - Vr H) sinv
  DBuf B2(&dev, (size_t)mn * chi * 8);
  contract(dev, m, view(T.p, T_F64, {mn, chi}, "ik"), Vrv, view(Hm.p, T_F64, {r, chi}, "qk"));
  HIP_CHECK(ctmk::launch_sub_sinv((const double*)Vbar.p, (const double*)T.p, mn, chi, sv, w, (double*)B2.p, dev.stream));
  // rhobar = Gm Vr^T + Ur[:, :chi] B2^T  (mn x mn)
  DBuf rb(&dev, (size_t)mn * mn * 8);
  TRef rbv = view(rb.p, T_F64, {mn, mn}, "ij");
  contract(dev, m, rbv, Gmv, TRef{Vr, T_F64, {mn, r}, {1, mn}, "jp"});
  contract(dev, m, rbv, TRef{Ur, T_F64, {mn, chi}, {1, mn}, "ik"}, view(B2.p, T_F64, {mn, chi}, "jk"), 1.0, 1);
  // Nbar += rhobar S, Sbar += rhobar^T N
  contract(dev, m, Nb, rbv, relabel(Sv, "ja"), 1.0, 1);
  contract(dev, m, relabel(Sb, "ja"), rbv, Nv, 1.0, 1);
}

// Frobenius normalisation of the updated tensors, batched.  While the tape
// records, the norms are kept and the adjoint is recorded.
void normalize_all(ctm_ctx* c, const std::vector<TRef>& ts) {
  Dev& dev = c->dev;
  const bool rec = c->tape.recording();
  std::shared_ptr<DBuf> norms;
  if (rec) {
    TapePause pause(dev);
    norms = std::make_shared<DBuf>(&dev, std::max<size_t>(ts.size(), 1) * 8);
  }
  DBuf work;   // the kernels' partial sums: not part of the recorded computation
  {
    TapePause pause(dev);
    work = DBuf(&dev, (size_t)ctmk::normalize_work_doubles(ctmk::NORM_MAX) * 8);
  }
  for (size_t s0 = 0; s0 < ts.size(); s0 += ctmk::NORM_MAX) {
    ctmk::NormList L;
    std::memset(&L, 0, sizeof(L));
    int cnt = 0;
    for (size_t i = s0; i < ts.size() && cnt < ctmk::NORM_MAX; ++i, ++cnt) {
      L.ptr[cnt] = ts[i].p;
      L.n[cnt] = ts[i].numel();
    }
    if (rec) L.norm_out = (double*)norms->p + s0;
    L.zero_flag = (int*)c->flag.p + 3;
    HIP_CHECK(ctmk::launch_normalize(c->st, L, cnt, (double*)work.p, dev.stream));
  }
  if (!rec) return;
  std::vector<TRef> keep = ts;
  c->tape.custom([c, keep, norms]() {
    Tape& tp = c->tape;
    for (size_t s0 = 0; s0 < keep.size(); s0 += ctmk::NORM_MAX) {
      ctmk::NormList Y, Yb;
      std::memset(&Y, 0, sizeof(Y));
      std::memset(&Yb, 0, sizeof(Yb));
      int cnt = 0;
      for (size_t i = s0; i < keep.size() && cnt < ctmk::NORM_MAX; ++i, ++cnt) {
        Y.ptr[cnt] = keep[i].p;
        Y.n[cnt] = keep[i].numel();
        Yb.ptr[cnt] = tp.adj_ptr(keep[i].p);
        Yb.n[cnt] = Y.n[cnt];
      }
      Y.norm_out = (double*)norms->p + s0;
      HIP_CHECK(ctmk::launch_normalize_backward(c->st, Y, Yb, cnt, c->dev.stream));
    }
  });
}

// One left move in frame f (Fig. CTMRG b): for every column step J, the
// projectors of all rows, then C1, T4, C4 of column J+1 for all rows.
void left_move(ctm_ctx* c, int f) {
  Dev& dev = c->dev;
  const int a = c->ny(f), b = c->nx(f);
  const int64_t chi = c->chi, maxkd = chi * c->max_leg();
  const int m = c->mode;
  for (int J = 0; J < b; ++J) {
    DBuf P64(&dev, (size_t)a * maxkd * chi * 8), Q64(&dev, (size_t)a * maxkd * chi * 8);
    DBuf Pst, Qst;
    if (c->st != T_F64) {
      Pst = DBuf(&dev, (size_t)a * maxkd * chi * 4);
      Qst = DBuf(&dev, (size_t)a * maxkd * chi * 4);
    }
    std::vector<int64_t> zd(a);
    for (int I = 0; I < a; ++I) zd[I] = c->site(f, I, J).dim[3];
    column_projectors(c, f, J, (double*)P64.p, (double*)Q64.p, maxkd);
    if (c->st != T_F64) {
      for (int I = 0; I < a; ++I) {
        int64_t n = chi * zd[I] * chi;
        double* P = (double*)P64.p + (size_t)I * maxkd * chi;
        double* Q = (double*)Q64.p + (size_t)I * maxkd * chi;
        copy_into(dev, view((float*)Pst.p + (size_t)I * maxkd * chi, T_F32, {n}, "q"), view(P, T_F64, {n}, "q"));
        copy_into(dev, view((float*)Qst.p + (size_t)I * maxkd * chi, T_F32, {n}, "q"), view(Q, T_F64, {n}, "q"));
      }
    }
    auto PQ = [&](DBuf& B64, DBuf& Bst, int I, const std::string& lab) {
      int Ii = ((I % a) + a) % a;
      void* base = c->st == T_F64 ? (void*)((double*)B64.p + (size_t)Ii * maxkd * chi)
                                  : (void*)((float*)Bst.p + (size_t)Ii * maxkd * chi);
      return view(base, c->st, {chi, zd[Ii], chi}, lab);
    };
    std::vector<TRef> outs;
    // rows are independent here: when not recorded, the odd ones go to the
    // second stream (their outputs are slots of the environment buffer, their
    // temporaries from the second stream's cache)
    const bool two = !c->tape.recording() && c->streams > 1 && a > 1;
    SideScope side_scope(c, two);
    for (int I = 0; I < a; ++I) {
      Dev& rd = two && (I & 1) ? c->side : dev;
      TRef s = c->site_t(f, I, J, "yxrz");
      // C1' = [C1 T1] P_{I-1}
      Tmp X1(&rd, c->st, {chi, s.dim[1], chi}, "axc");
      contract(rd, m, X1.t, c->slot(f, I, J, 0, "ab"), c->slot(f, I, J, 4, "bxc"));
      TRef C1n = c->out_slot(f, I, J + 1, 0, "kc");
      contract(rd, m, C1n, PQ(P64, Pst, I - 1, "axk"), X1.t);
      // T4' = Q_{I-1}^T [T4 s] P_I
      Tmp G1(&rd, c->st, {chi, chi, s.dim[1], s.dim[2], s.dim[3]}, "eaxrz");
      absorb_site(c, rd, m, G1.t, c->slot(f, I, J, 7, "eya"), f, I, J, "yxrz");
      Tmp G2(&rd, c->st, {chi, chi, s.dim[2], s.dim[3]}, "emrz");
      contract(rd, m, G2.t, PQ(Q64, Qst, I - 1, "axm"), G1.t);
      TRef T4n = c->out_slot(f, I, J + 1, 7, "krm");
      contract(rd, m, T4n, PQ(P64, Pst, I, "ezk"), G2.t);
      // C4' = [C4 T3] Q_I
      Tmp V1(&rd, c->st, {chi, s.dim[3], chi}, "cwa");
      contract(rd, m, V1.t, c->slot(f, I, J, 6, "cwb"), c->slot(f, I, J, 3, "ba"));
      TRef C4n = c->out_slot(f, I, J + 1, 3, "ck");
      contract(rd, m, C4n, V1.t, PQ(Q64, Qst, I, "awk"));
      outs.push_back(C1n);
      outs.push_back(T4n);
      outs.push_back(C4n);
    }
    side_scope.join();
    normalize_all(c, outs);
  }
}

const int MOVE_FRAMES[4] = {0, 2, 1, 3};   // left, right, up, down

int corner_count(const ctm_ctx* c) { return c->NY * c->NX * 4; }

// Singular values (descending, chi per corner) of every corner of the current
// environment, in the order positions (I, J) row-major, then C1..C4.  A failed
// rocSOLVER solve is counted in the context's solver flag.
void corner_svals(ctm_ctx* c, DBuf& sv) {
  Dev& dev = c->dev;
  const int64_t chi = c->chi;
  const int count = corner_count(c);
  DBuf Cs(&dev, (size_t)count * chi * chi * 8), E(&dev, (size_t)count * chi * 8);
  DBuf infos(&dev, (size_t)count * sizeof(int));
  sv = DBuf(&dev, (size_t)count * chi * 8);
  for (int p = 0; p < c->NY * c->NX; ++p)
    for (int k = 0; k < 4; ++k) {
      TRef src = view((char*)c->env.p + c->slot_off[(size_t)p * 8 + k] * type_size(c->st), c->st, {chi, chi}, "ab");
      copy_into(dev, view((double*)Cs.p + (size_t)(p * 4 + k) * chi * chi, T_F64, {chi, chi}, "ab"), src);
    }
  RB_CHECK(rocsolver_dgesvd_strided_batched(c->blas, rocblas_svect_none, rocblas_svect_none, (rocblas_int)chi,
                                            (rocblas_int)chi, (double*)Cs.p, (rocblas_int)chi, chi * chi,
                                            (double*)sv.p, chi, nullptr, 1, 0, nullptr, 1, 0, (double*)E.p, chi,
                                            rocblas_outofplace, (int*)infos.p, count));
  // info != 0: the bidiagonal iteration did not converge for that corner
  HIP_CHECK(ctmk::launch_flag_or((const int*)infos.p, count, (int*)c->flag.p + 1, dev.stream));
}

// Normalised corner spectra of the environment and their L1 change.
double spectra_delta(ctm_ctx* c) {
  Dev& dev = c->dev;
  const int64_t chi = c->chi;
  const int count = corner_count(c);
  DBuf sv;
  corner_svals(c, sv);
  if (!c->spec_cur.p) {
    c->spec_cur = DBuf(&dev, (size_t)count * chi * 8);
    c->spec_prev = DBuf(&dev, (size_t)count * chi * 8);
  }
  HIP_CHECK(ctmk::launch_spectra_delta((const double*)sv.p, chi, chi, (double*)c->spec_cur.p,
                                       c->have_prev ? (const double*)c->spec_prev.p : nullptr, count,
                                       (double*)c->dscal.p, dev.stream));
  double delta = 0;
  HIP_CHECK(hipMemcpyAsync(&delta, c->dscal.p, 8, hipMemcpyDeviceToHost, dev.stream));
  HIP_CHECK(hipStreamSynchronize(dev.stream));
  std::swap(c->spec_cur, c->spec_prev);
  bool first = !c->have_prev;
  c->have_prev = true;
  return first ? 1e300 : delta;
}

void check_flags(ctm_ctx* c) {
  int h[4] = {0, 0, 0, 0};
  HIP_CHECK(hipMemcpyAsync(h, c->flag.p, sizeof(h), hipMemcpyDeviceToHost, c->dev.stream));
  HIP_CHECK(hipStreamSynchronize(c->dev.stream));
  HIP_CHECK(hipMemsetAsync(c->flag.p, 0, sizeof(h), c->dev.stream));
  // a failed solve or an empty cut first: either is the cause of whatever
  // else went wrong after it
  if (h[1]) throw Error(CTM_ESOLVER, "SVD did not converge (" + std::to_string(h[1]) + " failed solves)");
  if (h[2])
    throw Error(CTM_ESOLVER, "empty cut: the bond density matrix of " + std::to_string(h[2]) +
                                 " cut(s) vanished to working precision (s_1 <= 1e-12 |N||S|), no projector exists");
  if (h[3]) throw Error(CTM_ESOLVER, "an updated environment tensor is zero (" + std::to_string(h[3]) + " tensors)");
  if (h[0]) throw Error(CTM_ENONFINITE, "non-finite value in the environment");
}

// ---------------------------------------------------------------------------
// 2x2 reduced density matrix of the plaquette with top-left PEPS site (px, py)
// (impurity tensors of Sec. II B).  The nested block is rows 2py..2py+3 and
// columns 2px..2px+3 with its border environment.  The four Y tensors are
// cut: the ket end of the physical line stays with the fused leg coming from
// K, the bra end is exposed on the B below.  X and cut Y tensors are pure
// relabellings of legs.
//
// Contraction order: each PEPS site of the plaquette with its corner and two
// pairs of edge tensors forms a quadrant tensor with two cuts (a chi leg and
// two D legs each) and its two open physical legs; the two upper quadrants
// are joined over their common cut, likewise the two lower ones, and the two
// halves are joined over both vertical cuts.  No intermediate carries more
// than two quadrants' worth of open legs, so the largest tensor is a half of
// (chi D^2)^2 d^4 entries (the column-by-column order carries a strip of
// chi^2 D^4 d^4 entries and more).  Result:
// rho[(k_TL k_TR k_BL k_BR), (b_TL b_TR b_BL b_BR)].
// Plaquette density matrix of the double-layer network (Eq. Tred with the
// physical indices of the four sites open), with top-left site (px, py).
// Each quadrant is one corner, its two edges and one site; the site's ket
// tensor and then its bra tensor are contracted into it one layer at a time
// (the D^2 legs of the edges split into ket and bra halves), so the open
// reduced tensor itself (D^8 d^2 entries) is never formed.  Then the upper
// and the lower pair of quadrants, then the two halves.
void plaquette_rdm_double(ctm_ctx* c, int px, int py, double* rho_out) {
  Dev& dev = c->dev;
  const int m = c->emode;
  const int est = c->est;
  std::deque<Tmp> conv;
  auto in_est = [&](const TRef& t) -> TRef {
    if (t.type == est) return t;
    conv.emplace_back(&dev, est, t.dim, t.lab);
    copy_into(dev, conv.back().t, t);
    return conv.back().t;
  };
  const int64_t D = c->D, d = c->d, nk = d * D * D * D * D;
  Labels Lb;
  auto L = [&](const std::string& n) { return Lb(n); };
  auto str = [](std::initializer_list<char> l) { return std::string(l); };
  auto env = [&](int r, int cc, int k, const std::string& lab) { return in_est(c->slot(0, py + r, px + cc, k, lab)); };
  auto site = [&](int r, int cc, const std::string& lab) {
    const int y = (py + r) % c->Ly, x = (px + cc) % c->Lx;
    const int t = c->pattern[(size_t)y * c->Lx + x];
    return in_est(view((double*)c->A64.p + (size_t)t * nk, T_F64, {d, D, D, D, D}, lab));
  };
  auto absorb = [&](Tmp& S, const TRef& X) {
    std::string out;
    for (char ch : S.t.lab) if (X.lab.find(ch) == std::string::npos) out += ch;
    std::vector<int64_t> dims;
    for (char ch : out) dims.push_back(S.t.dim[S.t.lab.find(ch)]);
    for (size_t q = 0; q < X.lab.size(); ++q)
      if (S.t.lab.find(X.lab[q]) == std::string::npos) { out += X.lab[q]; dims.push_back(X.dim[q]); }
    Tmp R(&dev, est, dims, out);
    contract(dev, m, R.t, S.t, X);
    S = std::move(R);
  };
  auto start = [&](const TRef& corner) {
    Tmp S(&dev, est, corner.dim, corner.lab);
    copy_into(dev, S.t, corner);
    return S;
  };
  // a D^2 leg of the running tensor split into its ket (major) and bra halves
  auto split = [&](Tmp& S, const std::string& fused, const std::string& ket, const std::string& bra) {
    S.t = split_axis(S.t, L(fused), D, D, L(ket), L(bra));
  };
  // one quadrant: corner slot kc with edge slots ke1 and ke2 at position
  // (r, cc); the site legs (l, u, r, d) are named ``legs``, with suffix k on
  // the ket tensor and b on the bra tensor; the two legs that meet the edges
  // (leg1, leg2) are split into those halves first
  auto quadrant = [&](int r, int cc, int kc, const std::string& cl, int ke1, const std::string& e1,
                      int ke2, const std::string& e2, const std::string& leg1, const std::string& leg2,
                      const std::array<std::string, 4>& legs, const std::string& open) {
    Tmp Q = start(env(r, cc, kc, cl));
    absorb(Q, env(r, cc, ke1, e1));
    absorb(Q, env(r, cc, ke2, e2));
    split(Q, leg1, leg1 + "k", leg1 + "b");
    split(Q, leg2, leg2 + "k", leg2 + "b");
    auto lab = [&](const std::string& suffix, const std::string& phys) {
      std::string o = str({L(phys)});
      for (const auto& n : legs) o += L(n + suffix);
      return o;
    };
    absorb(Q, site(r, cc, lab("k", "k" + open)));
    absorb(Q, site(r, cc, lab("b", "b" + open)));
    return Q;
  };
  // chi legs: top t0 t1 t2, right R0 R1 R2, bottom b0 b1 b2, left L0 L1 L2;
  // D^2 legs between the plaquette's sites: m0 (TL-TR), m1 (BL-BR), n0 (TL-BL), n1 (TR-BR);
  // D^2 legs to the environment: v0 v1 (top), e0 e1 (right), w0 w1 (bottom), f0 f1 (left)
  auto cl = [&](const char* a, const char* b) { return str({L(a), L(b)}); };
  auto el = [&](const char* a, const char* b, const char* e) { return str({L(a), L(b), L(e)}); };
  Tmp TL = quadrant(0, 0, 0, cl("L0", "t0"), 4, el("t0", "v0", "t1"), 7, el("L1", "f0", "L0"), "f0", "v0",
                    {"f0", "v0", "m0", "n0"}, "TL");
  Tmp TR = quadrant(0, 1, 1, cl("t2", "R0"), 4, el("t1", "v1", "t2"), 5, el("R0", "e0", "R1"), "v1", "e0",
                    {"m0", "v1", "e0", "n1"}, "TR");
  Tmp BL = quadrant(1, 0, 3, cl("b0", "L2"), 6, el("b1", "w0", "b0"), 7, el("L2", "f1", "L1"), "w0", "f1",
                    {"f1", "n0", "m1", "w0"}, "BL");
  Tmp BR = quadrant(1, 1, 2, cl("R2", "b2"), 5, el("R1", "e1", "R2"), 6, el("b2", "w1", "b1"), "e1", "w1",
                    {"m1", "n1", "e1", "w1"}, "BR");
  absorb(TL, TR.t);   // over t1 and the ket and bra halves of m0
  absorb(BL, BR.t);   // over b1 and m1
  std::string ol;
  for (const char* n : {"kTL", "kTR", "kBL", "kBR", "bTL", "bTR", "bBL", "bBR"}) ol += L(n);
  std::vector<int64_t> od(8, d);
  if (est == T_F64) {
    contract(dev, m, view(rho_out, T_F64, od, ol), TL.t, BL.t);
  } else {
    Tmp r32(&dev, est, od, ol);
    contract(dev, m, r32.t, TL.t, BL.t);
    copy_into(dev, view(rho_out, T_F64, od, ol), r32.t);
  }
}

void plaquette_rdm(ctm_ctx* c, int px, int py, double* rho_out) {
  if (c->layout) {
    plaquette_rdm_double(c, px, py, rho_out);
    return;
  }
  Dev& dev = c->dev;
  // the energy's own precision: its environment and site tensors are copied
  // to the energy's storage type first when that differs from the sweep's
  const int m = c->emode;
  const int est = c->est;
  std::deque<Tmp> conv;
  auto in_est = [&](const TRef& t) -> TRef {
    if (t.type == est) return t;
    conv.emplace_back(&dev, est, t.dim, t.lab);
    copy_into(dev, conv.back().t, t);
    return conv.back().t;
  };
  const int64_t D = c->D, d = c->d;
  const int r0 = 2 * py, c0 = 2 * px;
  Labels Lb;
  auto H = [&](int r, int cc) { return Lb("H" + std::to_string(r) + "," + std::to_string(cc)); };     // bond right of (r,cc)
  auto Hd = [&](int r, int cc) { return Lb("Hd" + std::to_string(r) + "," + std::to_string(cc)); };   // D part of a fused bond
  auto V = [&](int r, int cc) { return Lb("V" + std::to_string(r) + "," + std::to_string(cc)); };     // bond below (r,cc)
  auto chL = [&](int i) { return Lb("cL" + std::to_string(i)); };
  auto chR = [&](int i) { return Lb("cR" + std::to_string(i)); };
  auto chT = [&](int i) { return Lb("cT" + std::to_string(i)); };
  auto chB = [&](int i) { return Lb("cB" + std::to_string(i)); };
  const char* names[4] = {"TL", "TR", "BL", "BR"};
  auto kO = [&](int s) { return Lb(std::string("k") + names[s]); };
  auto bO = [&](int s) { return Lb(std::string("b") + names[s]); };
  auto str = [](std::initializer_list<char> l) { return std::string(l); };

  auto env = [&](int r, int cc, int k, const std::string& lab) { return in_est(c->slot(0, r0 + r, c0 + cc, k, lab)); };
  auto site = [&](int r, int cc, const std::string& lab) { return in_est(c->site_t(0, r0 + r, c0 + cc, lab)); };

  auto absorb = [&](Tmp& S, const TRef& X) {
    std::string out;
    for (char ch : S.t.lab) if (X.lab.find(ch) == std::string::npos) out += ch;
    std::vector<int64_t> dims;
    for (char ch : out) dims.push_back(S.t.dim[S.t.lab.find(ch)]);
    for (size_t q = 0; q < X.lab.size(); ++q)
      if (S.t.lab.find(X.lab[q]) == std::string::npos) { out += X.lab[q]; dims.push_back(X.dim[q]); }
    Tmp R(&dev, est, dims, out);
    contract(dev, m, R.t, S.t, X);
    S = std::move(R);
  };
  auto rename = [&](Tmp& S, char from, char to) {
    size_t i = S.t.lab.find(from);
    if (i == std::string::npos) throw Error(CTM_EINVAL, "rdm: missing label");
    S.t.lab[i] = to;
  };
  auto start = [&](const TRef& corner) {
    Tmp S(&dev, est, corner.dim, corner.lab);
    copy_into(dev, S.t, corner);
    return S;
  };
  // bra site with its fused up leg split (virtual U, physical = open bra index)
  auto bra = [&](int r, int cc, int s) {
    TRef Bt = site(r, cc, "lurd");
    Bt = split_axis(Bt, 'u', D, d, 'U', 'S');
    return relabel(Bt, str({H(r, cc - 1), V(r - 1, cc), bO(s), H(r, cc), V(r, cc)}));
  };
  // ket site with its fused right leg split (virtual R = Hd, physical = open ket index)
  auto ket_open = [&](int r, int cc, int s) {
    TRef Kt = site(r, cc, "lurd");
    Kt = split_axis(Kt, 'r', D, d, 'R', 'S');
    return relabel(Kt, str({H(r, cc - 1), V(r - 1, cc), Hd(r, cc), kO(s), V(r, cc)}));
  };

  // ---- TL quadrant: C1, T1(0,0), T4(0,0), K(0,0), T1(0,1), Y(0,1), T4(1,0), X(1,0), B(1,1)
  Tmp TL = start(env(0, 0, 0, str({chL(0), chT(0)})));
  absorb(TL, env(0, 0, 4, str({chT(0), V(-1, 0), chT(1)})));
  absorb(TL, env(0, 0, 7, str({chL(1), H(0, -1), chL(0)})));
  absorb(TL, site(0, 0, str({H(0, -1), V(-1, 0), H(0, 0), V(0, 0)})));
  absorb(TL, env(0, 1, 4, str({chT(1), V(-1, 1), chT(2)})));
  TL.t = split_axis(TL.t, H(0, 0), D, d, H(0, 1), kO(0));              // Y(0,1): ket index opened
  rename(TL, V(-1, 1), V(0, 1));
  absorb(TL, env(1, 0, 7, str({chL(2), H(1, -1), chL(1)})));
  rename(TL, H(1, -1), H(1, 0));                                       // X(1,0)
  rename(TL, V(0, 0), V(1, 0));
  absorb(TL, bra(1, 1, 0));                                            // B(1,1): bra index opened
  // ---- TR quadrant: C2, T1(0,3), T2(0,3), Y(0,3), T1(0,2), K(0,2), T2(1,3), B(1,3), X(1,2)
  Tmp TR = start(env(0, 3, 1, str({chT(4), chR(0)})));
  absorb(TR, env(0, 3, 4, str({chT(3), V(-1, 3), chT(4)})));
  absorb(TR, env(0, 3, 5, str({chR(0), H(0, 3), chR(1)})));
  rename(TR, H(0, 3), Hd(0, 2));                                       // Y(0,3): virtual part of K's leg
  rename(TR, V(-1, 3), V(0, 3));
  absorb(TR, env(0, 2, 4, str({chT(2), V(-1, 2), chT(3)})));
  absorb(TR, ket_open(0, 2, 1));                                       // K(0,2): ket index opened
  absorb(TR, env(1, 3, 5, str({chR(1), H(1, 3), chR(2)})));
  absorb(TR, bra(1, 3, 1));                                            // B(1,3)
  rename(TR, H(1, 2), H(1, 1));                                        // X(1,2)
  rename(TR, V(0, 2), V(1, 2));
  // ---- BL quadrant: C4, T4(3,0), T3(3,0), X(3,0), T4(2,0), K(2,0), T3(3,1), B(3,1), Y(2,1)
  Tmp BL = start(env(3, 0, 3, str({chB(0), chL(4)})));
  absorb(BL, env(3, 0, 7, str({chL(4), H(3, -1), chL(3)})));
  absorb(BL, env(3, 0, 6, str({chB(1), V(3, 0), chB(0)})));
  rename(BL, H(3, -1), H(3, 0));                                       // X(3,0)
  rename(BL, V(3, 0), V(2, 0));
  absorb(BL, env(2, 0, 7, str({chL(3), H(2, -1), chL(2)})));
  absorb(BL, site(2, 0, str({H(2, -1), V(1, 0), H(2, 0), V(2, 0)})));
  absorb(BL, env(3, 1, 6, str({chB(2), V(3, 1), chB(1)})));
  absorb(BL, bra(3, 1, 2));                                            // B(3,1)
  BL.t = split_axis(BL.t, H(2, 0), D, d, H(2, 1), kO(2));              // Y(2,1)
  rename(BL, V(2, 1), V(1, 1));
  // ---- BR quadrant: C3, T2(3,3), T3(3,3), B(3,3), T2(2,3), Y(2,3), T3(3,2), X(3,2), K(2,2)
  Tmp BR = start(env(3, 3, 2, str({chR(4), chB(4)})));
  absorb(BR, env(3, 3, 5, str({chR(3), H(3, 3), chR(4)})));
  absorb(BR, env(3, 3, 6, str({chB(4), V(3, 3), chB(3)})));
  absorb(BR, bra(3, 3, 3));                                            // B(3,3)
  absorb(BR, env(2, 3, 5, str({chR(2), H(2, 3), chR(3)})));
  rename(BR, H(2, 3), Hd(2, 2));                                       // Y(2,3)
  rename(BR, V(2, 3), V(1, 3));
  absorb(BR, env(3, 2, 6, str({chB(3), V(3, 2), chB(2)})));
  rename(BR, H(3, 2), H(3, 1));                                        // X(3,2)
  rename(BR, V(3, 2), V(2, 2));
  absorb(BR, ket_open(2, 2, 3));                                       // K(2,2)
  // ---- halves and the join
  absorb(TL, TR.t);   // over cT2, H(0,1), H(1,1)
  absorb(BL, BR.t);   // over cB2, H(2,1), H(3,1)
  std::string ol = str({kO(0), kO(1), kO(2), kO(3), bO(0), bO(1), bO(2), bO(3)});
  std::vector<int64_t> od(8, d);
  if (est == T_F64) {
    contract(dev, m, view(rho_out, T_F64, od, ol), TL.t, BL.t);
  } else {
    Tmp r32(&dev, est, od, ol);
    contract(dev, m, r32.t, TL.t, BL.t);
    copy_into(dev, view(rho_out, T_F64, od, ol), r32.t);
  }
}

// Energy per site (Eq. ExpH) from the current environment; while the tape
// records, the adjoint d E / d rho of the density matrices is recorded.
double energy_impl(ctm_ctx* c, const double* H_bond, int n_terms, const ctm_term* terms) {
  std::vector<std::pair<int, int>> plaq;
  std::vector<ctmk::EnergyTerm> et(n_terms);
  for (int i = 0; i < n_terms; ++i) {
    const ctm_term& t = terms[i];
    if (t.px < 0 || t.px >= c->Lx || t.py < 0 || t.py >= c->Ly || t.a < 0 || t.a > 3 || t.b < 0 || t.b > 3 || t.a == t.b)
      throw Error(CTM_EINVAL, "invalid term");
    int idx = -1;
    for (size_t q = 0; q < plaq.size(); ++q)
      if (plaq[q] == std::make_pair(t.px, t.py)) idx = (int)q;
    if (idx < 0) { idx = (int)plaq.size(); plaq.push_back({t.px, t.py}); }
    et[i].rho_index = idx; et[i].a = t.a; et[i].b = t.b; et[i].coef = t.coef;
  }
  const int64_t d4 = (int64_t)c->d * c->d * c->d * c->d, rsz = d4 * d4;
  if (plaq.empty()) return 0.0;
  c->rdm_buf = DBuf(&c->dev, (size_t)plaq.size() * rsz * 8);
  c->n_rdm = (int)plaq.size();
  for (size_t q = 0; q < plaq.size(); ++q)
    plaquette_rdm(c, plaq[q].first, plaq[q].second, (double*)c->rdm_buf.p + q * rsz);
  const bool rec = c->tape.recording();
  TapePause pause(c->dev);
  auto hb = std::make_shared<DBuf>(&c->dev, (size_t)d4 * 8);
  auto tb = std::make_shared<DBuf>(&c->dev, sizeof(ctmk::EnergyTerm) * std::max(n_terms, 1));
  auto bond = std::make_shared<DBuf>(&c->dev, (size_t)std::max(n_terms, 1) * 8);
  HIP_CHECK(hipMemcpyAsync(hb->p, H_bond, (size_t)d4 * 8, hipMemcpyHostToDevice, c->dev.stream));
  HIP_CHECK(hipMemcpyAsync(tb->p, et.data(), sizeof(ctmk::EnergyTerm) * n_terms, hipMemcpyHostToDevice, c->dev.stream));
  const double inv_sites = 1.0 / (c->Lx * c->Ly);
  HIP_CHECK(ctmk::launch_energy((const double*)c->rdm_buf.p, rsz, (const double*)hb->p,
                                (const ctmk::EnergyTerm*)tb->p, n_terms, c->d, inv_sites, (double*)c->dscal.p,
                                (double*)bond->p, c->dev.stream));
  HIP_CHECK(ctmk::launch_nonfinite(T_F64, c->dscal.p, 1, (int*)c->flag.p, c->dev.stream));
  double E = 0.0;
  HIP_CHECK(hipMemcpyAsync(&E, c->dscal.p, 8, hipMemcpyDeviceToHost, c->dev.stream));
  HIP_CHECK(hipStreamSynchronize(c->dev.stream));
  if (rec) {
    void* rho = c->rdm_buf.p;
    int nr = (int)plaq.size();
    c->tape.custom([c, rho, rsz, hb, tb, bond, n_terms, nr, inv_sites]() {
      HIP_CHECK(ctmk::launch_energy_backward((const double*)rho, rsz, (const double*)hb->p,
                                             (const ctmk::EnergyTerm*)tb->p, n_terms, c->d, inv_sites,
                                             (const double*)bond->p, nr, (double*)c->tape.adj_ptr(rho),
                                             c->dev.stream));
    });
  }
  return E;
}

// Adjoint of the site tensors of all frames (site_adj mirrors site_buf) added
// up into dE/dA[t][s][l][u][r][d] (float64, overwritten).
void sites_adjoint_to_A(ctm_ctx* c, const void* site_adj, double* grad) {
  Dev& dev = c->dev;
  const int d = c->d, D = c->D;
  const int64_t Dd = (int64_t)D * d, n4 = (int64_t)D * D * D * D, nk = (int64_t)d * n4, ny_ = (int64_t)d * d * n4;
  const int64_t per_frame = 2 * c->nt * nk + n4 + ny_;
  const size_t es = type_size(c->st);
  fill(dev, view(grad, T_F64, {c->nt * nk}, "q"), 0.0);
  const std::string lurd = "lurd";
  Tmp k0(&dev, T_F64, {D, D, D, d, D}, "lursd");
  Tmp b0(&dev, T_F64, {D, D, d, D, D}, "lusrd");
  for (int f = 0; f < 4; ++f) {
    std::string rl;
    for (int i = 0; i < 4; ++i) rl += lurd[(i + f) % 4];
    const char* fb = (const char*)site_adj + (size_t)f * per_frame * es;
    int64_t kd0[4] = {D, D, Dd, D}, bd0[4] = {D, Dd, D, D}, nk_[4], nb_[4];
    for (int i = 0; i < 4; ++i) { nk_[i] = kd0[(i + f) % 4]; nb_[i] = bd0[(i + f) % 4]; }
    for (int t = 0; t < c->nt; ++t) {
      TRef gA = view(grad + t * nk, T_F64, {d, D, D, D, D}, "slurd");
      copy_into(dev, view(k0.buf.p, T_F64, {kd0[0], kd0[1], kd0[2], kd0[3]}, lurd),
                view((void*)(fb + (size_t)(2 * t) * nk * es), c->st, {nk_[0], nk_[1], nk_[2], nk_[3]}, rl));
      copy_into(dev, gA, k0.t, true);
      copy_into(dev, view(b0.buf.p, T_F64, {bd0[0], bd0[1], bd0[2], bd0[3]}, lurd),
                view((void*)(fb + (size_t)(2 * t + 1) * nk * es), c->st, {nb_[0], nb_[1], nb_[2], nb_[3]}, rl));
      copy_into(dev, gA, b0.t, true);
    }
  }
}

// E and dE/dA of the energy after n sweeps from the current environment,
// which is held constant (the shortened chain of Sec. IV).  Checkpointing:
// the forward pass keeps one environment snapshot per sweep; the reverse
// pass recomputes one sweep at a time under the tape and propagates the
// environment adjoint back through it, so the tape never holds more than one
// sweep.  The environment is left at the result of the n sweeps.
// E after n sweeps from the current environment and dE/dA.  The last sweep
// and the energy are recorded on one tape during the forward pass (one
// sweep's tape takes a few GB at D = 6, chi = 72); the sweeps before it are run
// without a tape from snapshots of their starting environments and recomputed
// under the tape in reverse order (checkpointing at sweep granularity).
// Clears the context's projector-cache pointers when the scope ends (the
// caches are locals of the caller) and restores the projector SVD method:
// every sweep of a differentiated chain, the forward ones that the reverse
// pass recomputes included, takes the exact SVD, so that the recomputation
// follows the forward pass.
struct ProjCacheScope {
  ctm_ctx* c;
  int svd_method;
  explicit ProjCacheScope(ctm_ctx* cc) : c(cc), svd_method(cc->svd_method) { c->svd_method = 0; }
  ~ProjCacheScope() {
    c->pc_fill = nullptr;
    c->pc_use = nullptr;
    c->pc_pos = 0;
    c->svd_method = svd_method;
  }
};

// Adjoint buffers of the tensors the recorded sweeps and the energy read:
// the nested sites, or on the double-layer network the per-frame copies of A
// that the layered absorption reads and the float64 A of the density
// matrices.  Zeroed once, registered with every tape of a reverse pass.
struct SiteAdjoints {
  DBuf a, b;
  explicit SiteAdjoints(ctm_ctx* c) {
    Dev& dev = c->dev;
    const DBuf& src = c->layout ? c->a_frames : c->site_buf;
    a = DBuf(&dev, src.bytes);
    HIP_CHECK(hipMemsetAsync(a.p, 0, a.bytes, dev.stream));
    if (c->layout) {
      b = DBuf(&dev, c->A64.bytes);
      HIP_CHECK(hipMemsetAsync(b.p, 0, b.bytes, dev.stream));
    }
  }
  void reg(ctm_ctx* c) const {
    if (!c->layout) {
      c->tape.reg(c->site_buf.p, c->site_buf.bytes, a.p);
    } else {
      c->tape.reg(c->a_frames.p, c->a_frames.bytes, a.p);
      c->tape.reg(c->A64.p, c->A64.bytes, b.p);
    }
  }
  // dE/dA[t][s][l][u][r][d] (float64, overwritten)
  void to_A(ctm_ctx* c, double* grad) const {
    if (!c->layout) {
      sites_adjoint_to_A(c, a.p, grad);
      return;
    }
    Dev& dev = c->dev;
    const int64_t d = c->d, D = c->D, nk = d * D * D * D * D;
    const size_t es = type_size(c->st);
    HIP_CHECK(hipMemcpyAsync(grad, b.p, (size_t)c->nt * nk * 8, hipMemcpyDeviceToDevice, dev.stream));
    const std::string lurd = "lurd";
    for (int f = 0; f < 4; ++f) {
      std::string rl = "s";
      for (int q = 0; q < 4; ++q) rl += lurd[(q + f) % 4];
      for (int t = 0; t < c->nt; ++t)
        copy_into(dev, view(grad + t * nk, T_F64, {d, D, D, D, D}, "slurd"),
                  view((char*)a.p + (size_t)(f * c->nt + t) * nk * es, c->st, {d, D, D, D, D}, rl), true);
    }
  }
};

double energy_grad_impl(ctm_ctx* c, int n, const double* H_bond, int n_terms, const ctm_term* terms, double* grad) {
  Dev& dev = c->dev;
  const size_t eb = (size_t)c->env_elems * type_size(c->st);
  const size_t es = type_size(c->st);
  std::vector<DBuf> snap;
  // projector blocks of the sweeps the reverse pass recomputes (option proj_cache)
  std::vector<std::vector<ProjCacheStep>> pcache(c->proj_cache && n > 1 ? n - 1 : 0);
  ProjCacheScope pc_scope(c);
  for (int i = 0; i + 1 < n; ++i) {
    snap.emplace_back(&dev, eb);
    HIP_CHECK(hipMemcpyAsync(snap.back().p, c->env.p, eb, hipMemcpyDeviceToDevice, dev.stream));
    c->pc_fill = pcache.empty() ? nullptr : &pcache[i];
    for (int f : MOVE_FRAMES) left_move(c, f);
    c->pc_fill = nullptr;
  }
  DBuf final_env(&dev, eb);
  SiteAdjoints site_adj(c);
  DBuf env_adj(&dev, eb), env_adj2(&dev, eb);
  HIP_CHECK(hipMemsetAsync(env_adj.p, 0, eb, dev.stream));
  // the last sweep and the energy at its environment, on one tape
  c->tape.begin(&dev);
  site_adj.reg(c);
  c->tape.reg(c->env.p, eb, env_adj.p);
  if (n > 0)
    for (int f : MOVE_FRAMES) left_move(c, f);
  double E = energy_impl(c, H_bond, n_terms, terms);
  {
    // the environment after the sweep sits in the fresh buffers of the slots
    TapePause pause(dev);
    for (size_t idx = 0; idx < c->slot_ptr.size(); ++idx) {
      const int64_t ne = c->slot_elems(idx);
      copy_into(dev, view((char*)final_env.p + c->slot_off[idx] * es, c->st, {ne}, "q"),
                view(c->slot_ptr[idx], c->st, {ne}, "q"));
    }
    HIP_CHECK(ctmk::launch_nonfinite(c->st, final_env.p, c->env_elems, (int*)c->flag.p, dev.stream));
  }
  c->tape.backward();   // env_adj: dE / d(environment before the last sweep)
  c->tape.clear();
  c->reset_slot_ptrs();
  // earlier sweeps in reverse order, recomputed from their snapshots
  for (int i = n - 2; i >= 0; --i) {
    HIP_CHECK(hipMemcpyAsync(c->env.p, snap[i].p, eb, hipMemcpyDeviceToDevice, dev.stream));
    c->reset_slot_ptrs();
    HIP_CHECK(hipMemsetAsync(env_adj2.p, 0, eb, dev.stream));
    c->tape.begin(&dev);
    site_adj.reg(c);
    c->tape.reg(c->env.p, eb, env_adj2.p);
    c->pc_use = pcache.empty() ? nullptr : &pcache[i];
    c->pc_pos = 0;
    for (int f : MOVE_FRAMES) left_move(c, f);
    c->pc_use = nullptr;
    // seed: the adjoint of the environment after this sweep
    TapePause pause(dev);
    for (size_t idx = 0; idx < c->slot_ptr.size(); ++idx) {
      const int64_t ne = c->slot_elems(idx);
      void* seed = (char*)env_adj.p + c->slot_off[idx] * es;
      copy_into(dev, view(c->tape.adj_ptr(c->slot_ptr[idx]), c->st, {ne}, "q"), view(seed, c->st, {ne}, "q"), true);
    }
    c->tape.backward();
    c->tape.clear();
    if (!pcache.empty()) pcache[i].clear();
    std::swap(env_adj, env_adj2);
    c->reset_slot_ptrs();
  }
  HIP_CHECK(hipMemcpyAsync(c->env.p, final_env.p, eb, hipMemcpyDeviceToDevice, dev.stream));
  c->reset_slot_ptrs();
  c->have_prev = false;
  site_adj.to_A(c, grad);
  HIP_CHECK(ctmk::launch_nonfinite(T_F64, grad, (int64_t)c->nt * c->d * c->D * c->D * c->D * c->D, (int*)c->flag.p,
                                   dev.stream));
  HIP_CHECK(hipStreamSynchronize(dev.stream));
  return E;
}

double device_max_abs(ctm_ctx* c, int type, const void* a, const void* b, int64_t n) {
  HIP_CHECK(ctmk::launch_max_abs(type, a, b, n, (double*)c->dscal.p + 1, c->dev.stream));
  double v = 0.0;
  HIP_CHECK(hipMemcpyAsync(&v, (double*)c->dscal.p + 1, 8, hipMemcpyDeviceToHost, c->dev.stream));
  HIP_CHECK(hipStreamSynchronize(c->dev.stream));
  return v;
}

// dE/dA of the converged energy E(A) = E(env*(A), A), env* = f(env*, A) the
// fixed point of the sweep map f (Eq. AD taken at the fixed point, Sec. IV).
// Implicit differentiation gives dE/dA = dE/dA|_env + lam df/dA with
// lam = dE/denv + lam df/denv, summed as lam = mu_0 + mu_1 + ... (mu_{k+1} =
// mu_k df/denv).  One sweep from the current environment (which must be the
// fixed point entry by entry, as the gauge rules of the projectors and the
// normalisation make a converged one) and the energy after it are recorded
// once; the first reverse pass gives dE/dA|_env + mu_0 df/dA and mu_1, every
// further pass over the sweep's operations alone, seeded with mu_k, adds
// mu_k df/dA and gives mu_{k+1}, until max|mu_k| <= tol max|mu_1|.  The
// environment is left at the result of the recorded sweep.
double energy_grad_fp_impl(ctm_ctx* c, const double* H_bond, int n_terms, const ctm_term* terms, double* grad,
                           double tol, int max_iter, int* iters, double* gap, bool* converged) {
  Dev& dev = c->dev;
  const size_t eb = (size_t)c->env_elems * type_size(c->st);
  const size_t es = type_size(c->st);
  DBuf final_env(&dev, eb), mu(&dev, eb);
  SiteAdjoints site_adj(c);
  DBuf env_adj(&dev, eb);
  HIP_CHECK(hipMemsetAsync(env_adj.p, 0, eb, dev.stream));
  c->tape.begin(&dev);
  site_adj.reg(c);
  c->tape.reg(c->env.p, eb, env_adj.p);
  for (int f : MOVE_FRAMES) left_move(c, f);
  const size_t n_sweep_ops = c->tape.ops.size();
  double E = energy_impl(c, H_bond, n_terms, terms);
  {
    TapePause pause(dev);
    for (size_t idx = 0; idx < c->slot_ptr.size(); ++idx) {
      const int64_t ne = c->slot_elems(idx);
      copy_into(dev, view((char*)final_env.p + c->slot_off[idx] * es, c->st, {ne}, "q"),
                view(c->slot_ptr[idx], c->st, {ne}, "q"));
    }
    HIP_CHECK(ctmk::launch_nonfinite(c->st, final_env.p, c->env_elems, (int*)c->flag.p, dev.stream));
  }
  const double env_max = device_max_abs(c, c->st, c->env.p, nullptr, c->env_elems);
  *gap = env_max > 0 ? device_max_abs(c, c->st, final_env.p, c->env.p, c->env_elems) / env_max : 0.0;
  c->tape.backward();   // dE/dA|_env + mu_0 df/dA into site_adj; mu_1 into env_adj
  const double norm0 = device_max_abs(c, c->st, env_adj.p, nullptr, c->env_elems);
  int k = 0;
  double mk = norm0;
  while (k < max_iter && mk > tol * norm0) {
    HIP_CHECK(hipMemcpyAsync(mu.p, env_adj.p, eb, hipMemcpyDeviceToDevice, dev.stream));
    c->tape.zero_own_adjoints();
    HIP_CHECK(hipMemsetAsync(env_adj.p, 0, eb, dev.stream));
    {
      TapePause pause(dev);
      for (size_t idx = 0; idx < c->slot_ptr.size(); ++idx) {
        const int64_t ne = c->slot_elems(idx);
        copy_into(dev, view(c->tape.adj_ptr(c->slot_ptr[idx]), c->st, {ne}, "q"),
                  view((char*)mu.p + c->slot_off[idx] * es, c->st, {ne}, "q"));
      }
    }
    c->tape.backward_range(0, n_sweep_ops);   // += mu_k df/dA into site_adj; mu_{k+1} into env_adj
    ++k;
    mk = device_max_abs(c, c->st, env_adj.p, nullptr, c->env_elems);
  }
  *iters = k;
  c->tape.clear();
  HIP_CHECK(hipMemcpyAsync(c->env.p, final_env.p, eb, hipMemcpyDeviceToDevice, dev.stream));
  c->reset_slot_ptrs();
  c->have_prev = false;
  site_adj.to_A(c, grad);
  HIP_CHECK(ctmk::launch_nonfinite(T_F64, grad, (int64_t)c->nt * c->d * c->D * c->D * c->D * c->D, (int*)c->flag.p,
                                   dev.stream));
  HIP_CHECK(hipStreamSynchronize(dev.stream));
  *converged = mk <= tol * norm0;
  return E;
}

int fail(ctm_ctx* c, const Error& e) {
  if (c) c->err = e.what();
  else g_init_error = e.what();
  return e.code;
}

}  // namespace

// =============================================================================
extern "C" {

}  // extern "C"

namespace {

int init_impl(ctm_ctx** out, const double* A, int d, int D, int chi, int Lx, int Ly, const int* pattern,
              int n_tensors, int precision, void* stream, int layout) {
  if (!out) { g_init_error = "out is NULL"; return CTM_EINVAL; }
  *out = nullptr;
  ctm_ctx* c = nullptr;
  try {
    if (!A || !pattern || d < 1 || D < 1 || Lx < 1 || Ly < 1 || n_tensors < 1)
      throw Error(CTM_EINVAL, "invalid dimensions or NULL pointer");
    if (!layout && (int64_t)chi < (int64_t)D * d) throw Error(CTM_EINVAL, "chi must be at least D*d");
    if (layout && (int64_t)chi < (int64_t)D * D) throw Error(CTM_EINVAL, "chi must be at least D*D");
    if (precision < CTM_FP64 || precision > CTM_MIXED) throw Error(CTM_EINVAL, "unknown precision");
    for (int i = 0; i < Lx * Ly; ++i)
      if (pattern[i] < 0 || pattern[i] >= n_tensors) throw Error(CTM_EINVAL, "pattern id out of range");
    c = new ctm_ctx();
    c->dev.stream = (hipStream_t)stream;
    c->d = d; c->D = D; c->chi = chi; c->Lx = Lx; c->Ly = Ly; c->nt = n_tensors; c->prec = precision;
    c->layout = layout;
    c->NY = layout ? Ly : 2 * Ly; c->NX = layout ? Lx : 2 * Lx;
    c->pattern.assign(pattern, pattern + Lx * Ly);
    c->st = (precision == CTM_FP64 || precision == CTM_MIXED) ? T_F64 : T_F32;
    c->mode = precision == CTM_BF16 ? ctmk::MODE_BF16 : (precision == CTM_FP32 ? ctmk::MODE_F32 : ctmk::MODE_F64);
    // CTM_MIXED: the sweep in FP64, the energy's contractions (and their
    // adjoints) in FP32 on the matrix cores
    c->est = precision == CTM_MIXED ? T_F32 : c->st;
    c->emode = precision == CTM_MIXED ? ctmk::MODE_F32 : c->mode;
    if (rocblas_create_handle(&c->blas) != rocblas_status_success) throw Error(CTM_EHIP, "rocblas_create_handle failed");
    RB_CHECK(rocblas_set_stream(c->blas, c->dev.stream));
    hipStream_t side = nullptr;
    HIP_CHECK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    c->side.stream = side;
    HIP_CHECK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    c->flag = DBuf(&c->dev, 64);
    c->dscal = DBuf(&c->dev, 64);
    HIP_CHECK(hipMemsetAsync(c->flag.p, 0, 64, c->dev.stream));
    int64_t nA = (int64_t)n_tensors * d * D * D * D * D;
    c->A64 = DBuf(&c->dev, (size_t)nA * 8);
    HIP_CHECK(hipMemcpyAsync(c->A64.p, A, (size_t)nA * 8, hipMemcpyDeviceToDevice, c->dev.stream));
    build_layout(c);
    c->env = DBuf(&c->dev, (size_t)c->env_elems * type_size(c->st));
    c->reset_slot_ptrs();
    build_sites(c);
    init_env(c);
    HIP_CHECK(hipStreamSynchronize(c->dev.stream));
    *out = c;
    return CTM_OK;
  } catch (const Error& e) {
    g_init_error = e.what();
    if (c) ctm_free(c);
    return e.code;
  } catch (const std::exception& e) {
    g_init_error = e.what();
    if (c) ctm_free(c);
    return CTM_EHIP;
  }
}

}  // namespace

extern "C" {

int ctm_init(ctm_ctx** out, const double* A, int d, int D, int chi, int Lx, int Ly, const int* pattern,
             int n_tensors, int precision, void* stream) {
  return init_impl(out, A, d, D, chi, Lx, Ly, pattern, n_tensors, precision, stream, 0);
}

int ctm_init_double_layer(ctm_ctx** out, const double* A, int d, int D, int chi, int Lx, int Ly, const int* pattern,
                          int n_tensors, int precision, void* stream) {
  return init_impl(out, A, d, D, chi, Lx, Ly, pattern, n_tensors, precision, stream, 1);
}

int ctm_set_tensors(ctm_ctx* c, const double* A) {
  if (!c || !A) return CTM_EINVAL;
  try {
    int64_t nA = (int64_t)c->nt * c->d * c->D * c->D * c->D * c->D;
    HIP_CHECK(hipMemcpyAsync(c->A64.p, A, (size_t)nA * 8, hipMemcpyDeviceToDevice, c->dev.stream));
    build_sites(c);
    return CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

int ctm_reset_env(ctm_ctx* c) {
  if (!c) return CTM_EINVAL;
  try { init_env(c); return CTM_OK; } catch (const Error& e) { return fail(c, e); }
}

int64_t ctm_env_size(const ctm_ctx* c) { return c ? c->env_elems : 0; }

int ctm_set_env(ctm_ctx* c, const double* env) {
  if (!c || !env) return CTM_EINVAL;
  try {
    copy_into(c->dev, view(c->env.p, c->st, {c->env_elems}, "e"), view((void*)env, T_F64, {c->env_elems}, "e"));
    c->have_prev = false;
    return CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

int ctm_get_env(ctm_ctx* c, double* env) {
  if (!c || !env) return CTM_EINVAL;
  try {
    copy_into(c->dev, view(env, T_F64, {c->env_elems}, "e"), view(c->env.p, c->st, {c->env_elems}, "e"));
    HIP_CHECK(hipStreamSynchronize(c->dev.stream));
    return CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

int ctm_sweep(ctm_ctx* c, int max_sweeps, double tol, int* sweeps_done, double* delta) {
  if (!c || max_sweeps < 0) return CTM_EINVAL;
  try {
    double dl = -1.0;
    int n = 0;
    const size_t eb = (size_t)c->env_elems * type_size(c->st);
    // conv_rdm: the plaquette density matrices of every plaquette of the cell,
    // each divided by its trace, of the environment the call starts from and
    // after every sweep
    const bool by_rdm = tol > 0 && c->conv_rdm;
    const int64_t d4 = (int64_t)c->d * c->d * c->d * c->d, rsz = d4 * d4, nplaq = (int64_t)c->Lx * c->Ly;
    auto all_rdms = [&](DBuf& out) {
      if (!out.p) out = DBuf(&c->dev, (size_t)nplaq * rsz * 8);
      for (int py = 0; py < c->Ly; ++py)
        for (int px = 0; px < c->Lx; ++px)
          plaquette_rdm(c, px, py, (double*)out.p + ((int64_t)py * c->Lx + px) * rsz);
      HIP_CHECK(ctmk::launch_rdm_normalize((double*)out.p, (int)nplaq, d4, c->dev.stream));
    };
    if (by_rdm) all_rdms(c->rdm_a);
    if (tol > 0 && !by_rdm && c->conv_env && !c->env_prev.p) c->env_prev = DBuf(&c->dev, eb);
    // the first delta compares with the spectra of the environment the call starts from
    if (tol > 0 && !by_rdm && !c->conv_env && !c->have_prev) (void)spectra_delta(c);
    for (n = 1; n <= max_sweeps; ++n) {
      if (tol > 0 && !by_rdm && c->conv_env)
        HIP_CHECK(hipMemcpyAsync(c->env_prev.p, c->env.p, eb, hipMemcpyDeviceToDevice, c->dev.stream));
      for (int f : MOVE_FRAMES) left_move(c, f);
      if (c->check_finite)
        HIP_CHECK(ctmk::launch_nonfinite(c->st, c->env.p, c->env_elems, (int*)c->flag.p, c->dev.stream));
      if (tol > 0) {
        if (by_rdm) {
          all_rdms(c->rdm_b);
          dl = device_max_abs(c, T_F64, c->rdm_b.p, c->rdm_a.p, nplaq * rsz);
          std::swap(c->rdm_a, c->rdm_b);
        } else if (c->conv_env) {
          const double mx = device_max_abs(c, c->st, c->env_prev.p, nullptr, c->env_elems);
          dl = mx > 0 ? device_max_abs(c, c->st, c->env.p, c->env_prev.p, c->env_elems) / mx : 1e300;
        } else {
          dl = spectra_delta(c);
        }
        check_flags(c);
        if (dl < tol) break;
      }
    }
    if (n > max_sweeps) n = max_sweeps;
    if (tol <= 0) check_flags(c);
    if (sweeps_done) *sweeps_done = n;
    if (delta) *delta = dl;
    return (tol > 0 && !(dl < tol)) ? CTM_ENOTCONV : CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

int ctm_corner_spectra(ctm_ctx* c, double* out, int64_t capacity, int64_t* n_written) {
  if (!c) return CTM_EINVAL;
  const int64_t total = (int64_t)corner_count(c) * c->chi;
  if (n_written) *n_written = 0;
  if (!out) {
    if (n_written) *n_written = total;
    return CTM_OK;
  }
  if (capacity < total) return fail(c, Error(CTM_EINVAL, "capacity below the number of corner spectrum values (4 chi per cell position)"));
  try {
    DBuf sv, norm(&c->dev, (size_t)total * 8);
    corner_svals(c, sv);
    HIP_CHECK(ctmk::launch_spectra_delta((const double*)sv.p, c->chi, c->chi, (double*)norm.p, nullptr,
                                         corner_count(c), (double*)c->dscal.p, c->dev.stream));
    HIP_CHECK(hipMemcpyAsync(out, norm.p, (size_t)total * 8, hipMemcpyDeviceToHost, c->dev.stream));
    check_flags(c);
    if (n_written) *n_written = total;
    return CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

int ctm_energy(ctm_ctx* c, const double* H_bond, int n_terms, const ctm_term* terms, double* E) {
  if (!c || !H_bond || (n_terms > 0 && !terms) || !E) return CTM_EINVAL;
  try {
    *E = energy_impl(c, H_bond, n_terms, terms);
    check_flags(c);
    return CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

int ctm_energy_grad(ctm_ctx* c, const double* A, int n_sweeps, const double* H_bond, int n_terms,
                    const ctm_term* terms, double* E, double* dEdA) {
  if (!c || !H_bond || (n_terms > 0 && !terms) || !E || !dEdA || n_sweeps < 0) return CTM_EINVAL;
  try {
    if (A) {
      int64_t nA = (int64_t)c->nt * c->d * c->D * c->D * c->D * c->D;
      HIP_CHECK(hipMemcpyAsync(c->A64.p, A, (size_t)nA * 8, hipMemcpyDeviceToDevice, c->dev.stream));
      build_sites(c);
    }
    *E = energy_grad_impl(c, n_sweeps, H_bond, n_terms, terms, dEdA);
    check_flags(c);
    return CTM_OK;
  } catch (const Error& e) {
    c->tape.clear();
    c->reset_slot_ptrs();
    return fail(c, e);
  }
}

int ctm_energy_grad_fp(ctm_ctx* c, const double* A, double tol, int max_iter, const double* H_bond, int n_terms,
                       const ctm_term* terms, double* E, double* dEdA, int* iters, double* gap) {
  if (!c || !H_bond || (n_terms > 0 && !terms) || !E || !dEdA || !(tol >= 0) || max_iter < 0) return CTM_EINVAL;
  try {
    if (A) {
      int64_t nA = (int64_t)c->nt * c->d * c->D * c->D * c->D * c->D;
      HIP_CHECK(hipMemcpyAsync(c->A64.p, A, (size_t)nA * 8, hipMemcpyDeviceToDevice, c->dev.stream));
      build_sites(c);
    }
    int k = 0;
    double g = 0.0;
    bool conv = false;
    *E = energy_grad_fp_impl(c, H_bond, n_terms, terms, dEdA, tol, max_iter, &k, &g, &conv);
    if (iters) *iters = k;
    if (gap) *gap = g;
    check_flags(c);
    return conv ? CTM_OK : CTM_ENOTCONV;
  } catch (const Error& e) {
    c->tape.clear();
    c->reset_slot_ptrs();
    return fail(c, e);
  }
}

int ctm_last_rdms(ctm_ctx* c, double* rho, int capacity, int* n) {
  if (!c || !rho || !n) return CTM_EINVAL;
  try {
    const int64_t d4 = (int64_t)c->d * c->d * c->d * c->d, rsz = d4 * d4;
    int k = std::min(capacity, c->n_rdm);
    if (k > 0) HIP_CHECK(hipMemcpyAsync(rho, c->rdm_buf.p, (size_t)k * rsz * 8, hipMemcpyDeviceToHost, c->dev.stream));
    HIP_CHECK(hipStreamSynchronize(c->dev.stream));
    *n = c->n_rdm;
    return CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

int ctm_observables(ctm_ctx* c, double* out, int capacity, int* n) {
  if (!c || !out || !n || capacity < 0) return CTM_EINVAL;
  try {
    if (c->d != 2) throw Error(CTM_EINVAL, "ctm_observables: spin-1/2 sites (d = 2) only");
    const int k = std::min(capacity, c->n_rdm);
    DBuf o;
    if (k > 0) {
      o = DBuf(&c->dev, (size_t)k * CTM_N_OBS * 8);
      HIP_CHECK(ctmk::launch_observables((const double*)c->rdm_buf.p, 256, k, (double*)o.p, c->dev.stream));
      HIP_CHECK(hipMemcpyAsync(out, o.p, (size_t)k * CTM_N_OBS * 8, hipMemcpyDeviceToHost, c->dev.stream));
    }
    HIP_CHECK(hipStreamSynchronize(c->dev.stream));
    *n = c->n_rdm;
    return CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

int ctm_set_option(ctm_ctx* c, const char* key, double value) {
  if (!c || !key) return CTM_EINVAL;
  std::string k(key);
  if (k == "svd_cutoff" && value >= 0) c->cutoff = value;
  else if (k == "proj_cache" && (value == 0 || value == 1)) c->proj_cache = (int)value;
  else if (k == "lorentz_eta" && value >= 0) c->eta = value;
  else if (k == "check_finite") c->check_finite = value != 0;
  else if (k == "streams" && (value == 1 || value == 2)) c->streams = (int)value;
  else if (k == "rowmajor_bf16") ctmk::g_rowmajor_path = value != 0;
  else if (k == "rowmajor_f64") ctmk::g_rowmajor_f64 = value != 0;
  else if (k == "rowmajor_f32") ctmk::g_rowmajor_f32 = value != 0;
  else if (k == "jacobi_one_launch") c->jacobi_one_launch = value != 0;
  else if (k == "jacobi_cooperative") c->jacobi_coop = value != 0;
  else if (k == "svd_method" && (value == 0 || value == 1)) c->svd_method = (int)value;
  else if (k == "conv_env" && (value == 0 || value == 1)) c->conv_env = (int)value;
  else if (k == "conv_rdm" && (value == 0 || value == 1)) c->conv_rdm = (int)value;
  else if (k == "svd_oversample" && value >= 0 && value <= 4096) c->rsvd_oversample = (int)value;
  else if (k == "svd_power" && value >= 0 && value <= 16) c->rsvd_power = (int)value;
  else if (k == "svd_seed" && value >= 0 && value < 9007199254740992.0) c->rsvd_seed = (uint64_t)value;
  else if (k == "energy_precision" && (value == CTM_FP64 || value == CTM_FP32 || value == CTM_BF16)) {
    c->est = value == CTM_FP64 ? T_F64 : T_F32;
    c->emode = value == CTM_BF16 ? ctmk::MODE_BF16 : (value == CTM_FP32 ? ctmk::MODE_F32 : ctmk::MODE_F64);
  }
  else if (k == "jacobi_max_sweeps" && value >= 1 && value <= 1000) c->jacobi_max_sweeps = (int)value;
  else if (k == "qr_fused_vy") g_qr_fused_vy = value != 0;
  else if (k == "qr_one_update") g_qr_one_update = value != 0;
  else { c->err = "unknown option or bad value: " + k; return CTM_EINVAL; }
  return CTM_OK;
}

int ctm_set_allocator(ctm_ctx* c, ctm_alloc_fn alloc, ctm_free_fn free_fn, void* user) {
  if (!c) return CTM_EINVAL;
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    c->err = "ctm_set_allocator: alloc and free must both be given or both be NULL";
    return CTM_EINVAL;
  }
  Dev::UserAlloc ua;
  ua.alloc = alloc;
  ua.free = free_fn;
  ua.user = user;
  c->dev.ua = ua;
  c->side.ua = ua;
  return CTM_OK;
}

int ctm_profile_begin(ctm_ctx* c) {
  if (!c) return CTM_EINVAL;
  try {
    HIP_CHECK(hipStreamSynchronize(c->dev.stream));
    g_counters.reset_timing();
    g_counters.timing = true;
    return CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

int ctm_profile_end(ctm_ctx* c, double* kernel_ms, double* kernel_flops, int64_t* launches) {
  if (!c) return CTM_EINVAL;
  try {
    g_counters.timing = false;
    double ms[N_FAMILIES];
    g_counters.collect_ms(ms);
    for (int i = 0; i < N_FAMILIES; ++i) {
      if (kernel_ms) kernel_ms[i] = ms[i];
      if (kernel_flops) kernel_flops[i] = g_counters.mode_flops[i];
      if (launches) launches[i] = g_counters.mode_launches[i];
    }
    g_counters.reset_timing();
    return CTM_OK;
  } catch (const Error& e) { return fail(c, e); }
}

const char* ctm_last_error(const ctm_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

void ctm_free(ctm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->dev.stream);
  {
    ctm_ctx* t = c;
    t->A64.reset(); t->site_buf.reset(); t->env.reset(); t->spec_prev.reset(); t->spec_cur.reset();
    t->dscal.reset(); t->rdm_buf.reset(); t->flag.reset(); t->env_prev.reset(); t->a_frames.reset(); t->rdm_a.reset(); t->rdm_b.reset();
  }
  c->tape.clear();
  c->dev.release();
  (void)hipStreamSynchronize(c->dev.stream);
  if (c->side.stream) {
    (void)hipStreamSynchronize(c->side.stream);
    c->side.release();
    (void)hipStreamSynchronize(c->side.stream);
    (void)hipStreamDestroy(c->side.stream);
    c->side.stream = nullptr;
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->blas) rocblas_destroy_handle(c->blas);
  delete c;
}

}  // extern "C"
