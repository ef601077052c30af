// Serving loop: continuous batching of independent solves on one GPU.
//
// A persistent host thread owns the device work.  Each turn it
//   1. admits queued requests while slots and the memory budget allow
//      (request vectors are carved from one pool allocated when the server
//      starts, so admission and retirement never allocate or free device
//      memory), builds or reuses the request's operator (set up once per
//      problem, mesh and degree, then kept resident) and starts its MINRES
//      state;
//   2. runs ONE MINRES step for every active request: one ragged operator
//      launch per (problem, degree) group carrying the first half of the
//      fused step, then one ragged launch of the second half over all active
//      requests;
//   3. every few steps reads all Krylov states back, retires converged
//      requests (true FP64 residual, optional copy of the solution) and
//      returns their vectors to the pool, so queued requests can enter the
//      mix.
// With the block preconditioner (mixed Poisson) each step adds one ragged
// batch of preconditioner applies over the requests that use it.
// Every request keeps its own blocks, partial sums and scalar state, so its
// iterates are the same whether it runs alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "gym_internal.hpp"
#include "kernels.hpp"
#include "krylov.hpp"
#include "schur.hpp"

using namespace gym;

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kStages = 4;      // ring of per-step parameter uploads
constexpr int kCheckEvery = 8;  // steps between reads of the Krylov states
constexpr int kMaxGroups = 8;   // (problem, degree) pairs

struct OpEntry {
  gym_mesh* mesh = nullptr;
  gym_op* op = nullptr;
  SchurPrec* schur = nullptr;  // set up on the first request that needs it
  int refs = 0;
  size_t bytes = 0;
};

// First-fit pool over one device allocation: blocks are carved at admission
// and given back at retirement (adjacent free blocks merge), so the loop
// thread allocates and frees no device memory for requests (hipFree would
// synchronise the device under the running mix).
class Pool {
 public:
  static constexpr size_t kAlign = 256;
  void reset(char* base, size_t size) {
    base_ = base;
    free_.clear();
    if (size) free_[0] = size;
  }
  char* base() const { return base_; }
  static size_t round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
  bool fits(size_t bytes) const {
    bytes = round(bytes);
    for (const auto& f : free_)
      if (f.second >= bytes) return true;
    return false;
  }
  char* take(size_t bytes) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, left = it->second - bytes;
      free_.erase(it);
      if (left) free_[off + bytes] = left;
      return base_ + off;
    }
    return nullptr;
  }
  void give(char* p, size_t bytes) {
    size_t off = (size_t)(p - base_);
    bytes = round(bytes);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }

 private:
  char* base_ = nullptr;
  std::map<size_t, size_t> free_;  // offset -> size
};

struct Pending {
  uint64_t id;
  gym_request req;
  std::vector<double> rhs;
  Clock::time_point t0;
  int64_t n;
  size_t bytes;       // vectors + operator (budget check)
  size_t slot_bytes;  // vectors (pool block)
  int64_t np;         // cell unknowns (block preconditioner work vectors)
};

struct Slot {
  uint64_t id;
  int problem, degree;
  bool want_x;
  Clock::time_point t0;
  OpEntry* op;
  long long n;
  int nb;   // blocks of the vector kernel
  int npa;  // operator workgroups of the last step
  size_t bytes;
  SchurPrec* schur;  // block preconditioner, or null (Jacobi)
  double *sw0, *sw1;  // its work vectors (cell block), in the slot's own memory
  double *b, *x;
  double *r1, *r2, *y, *z, *zp, *w, *w1, *w2;  // current roles
  double *pa, *pb[2], *pc[2], *alfa[2];         // step partials (two alternating sets)
  double *scratch, *sums;                       // residual norms
  int par;       // partial set written last
  bool pending;  // a MINRES step awaits closing
  void* mem;
  int sidx;  // state pair index
  int it;    // steps launched
  int tighten;    // residual re-checks so far
  double* R0[3];  // initial (r1, r2, y) buffers
  double* Z0[2];  // initial (z, zp)
  double* W0[3];  // initial (w, w1, w2) buffers
};

struct Done {
  gym_result res;
  std::vector<double> x;
};

int64_t request_ndofs(const gym_request& r) {
  int64_t nel[3] = {r.nel, r.nel, r.nel};
  SpaceDesc a, b;
  if (r.problem == GYM_MIXED_POISSON) {
    a = make_space_desc(GYM_HDIV, 3, nel, r.degree, GYM_BC_NATURAL);
    b = make_space_desc(GYM_L2, 3, nel, r.degree, GYM_BC_NATURAL);
  } else {
    a = make_space_desc(GYM_H1, 3, nel, r.degree, GYM_BC_ESSENTIAL);
    b = make_space_desc(GYM_HCURL, 3, nel, r.degree, GYM_BC_ESSENTIAL);
  }
  return a.ndofs + b.ndofs;
}

// Device doubles of a slot: 10 vectors, the operator's partial sums (at
// most one workgroup per element), two sets of step partials, the residual
// scratch.
size_t slot_doubles(int64_t n, int nel, int nb) {
  return 10 * (size_t)n + (size_t)nel * nel * nel + 4 * (size_t)nb + 2 + (size_t)nb + 2;
}

// slot buffers plus the operator's preconditioner
size_t request_bytes(int64_t n, int nel, int ncu) {
  return sizeof(double) * (slot_doubles(n, nel, vec_grid(n, ncu)) + (size_t)n);
}

}  // namespace

struct gym_server {
  gym_ctx* ctx = nullptr;
  gym_serve_opts opts{};
  hipStream_t stream = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Pending> queue;
  std::unordered_map<uint64_t, Done> done;
  std::unordered_map<uint64_t, int> pending;
  std::vector<Slot*> active;
  size_t bytes_used = 0;
  bool stopping = false;
  uint64_t next_id = 1;
  std::map<std::tuple<int, int, int>, OpEntry*> ops;
  MinresState* d_states = nullptr;
  MinresState* h_states = nullptr;
  std::vector<int> free_sidx;
  OpParams* plist_h[kStages] = {};
  OpParams* plist_d[kStages] = {};
  int* bst_h[kStages] = {};
  int* bst_d[kStages] = {};
  MrItem* items_h[kStages] = {};
  MrItem* items_d[kStages] = {};
  SchurItem* sitems_h[kStages] = {};  // block preconditioner batch
  SchurItem* sitems_d[kStages] = {};
  int* stab_h[kStages] = {};          // its block tables: elementwise, then axes 0..2
  int* stab_d[kStages] = {};
  int* ibst_h[kStages] = {};
  int* ibst_d[kStages] = {};
  hipEvent_t ev[kStages] = {};
  int stage = 0;
  void* pool_mem = nullptr;
  Pool pool;
  int fatal = 0;
  std::string fatal_msg;
};

namespace {

int record_fatal(gym_server* s, int code) {
  s->fatal = code;
  s->fatal_msg = gym_last_error();
  return code;
}

OpEntry* get_op(gym_server* s, int problem, int nel, int degree, int* rc) {
  auto key = std::make_tuple(problem, nel, degree);
  auto it = s->ops.find(key);
  if (it != s->ops.end()) return it->second;
  OpEntry* e = new OpEntry;
  int64_t n3[3] = {nel, nel, nel};
  *rc = gym_mesh_create(s->ctx, 3, n3, nullptr, nullptr, nullptr, &e->mesh);
  if (*rc) {
    delete e;
    return nullptr;
  }
  *rc = gym_op_create(s->ctx, problem, e->mesh, degree, &e->op);
  if (*rc) {
    gym_mesh_destroy(e->mesh);
    delete e;
    return nullptr;
  }
  e->bytes = sizeof(double) * (size_t)gym_op_ndofs(e->op);
  s->ops[key] = e;
  s->bytes_used += e->bytes;
  return e;
}

// free cached operators nobody uses until `need` more bytes fit
void evict_ops(gym_server* s, size_t need) {
  for (auto it = s->ops.begin(); it != s->ops.end() && s->bytes_used + need > (size_t)s->opts.mem_budget;) {
    OpEntry* e = it->second;
    if (e->refs == 0) {
      s->bytes_used -= e->bytes;
      gym_op_destroy(e->op);  // frees the preconditioner kept with it
      gym_mesh_destroy(e->mesh);
      delete e;
      it = s->ops.erase(it);
    } else {
      ++it;
    }
  }
}

// device bytes of a preconditioner's factors and work vectors
size_t schur_bytes(const SchurPrec& P) {
  size_t f = 0;
  for (int a = 0; a < 3; ++a) f += (size_t)P.m[a] * P.m[a];
  return sizeof(double) * ((size_t)P.ns + P.m[0] + P.m[1] + P.m[2] + 2 * f) + sizeof(float) * 2 * f + P.work_bytes;
}

int admit(gym_server* s, Pending& p) {
  int rc = 0;
  OpEntry* e = get_op(s, p.req.problem, p.req.nel, p.req.degree, &rc);
  if (!e) return rc;
  if (s->opts.precond == GYM_PRECOND_SCHUR && !e->schur) {
    if (int rc2 = ensure_schur(e->op, 1, &e->schur)) return rc2;
    const size_t b = schur_bytes(*e->schur);
    e->bytes += b;
    s->bytes_used += b;
  }
  char* mem = s->pool.take(p.slot_bytes);
  if (!mem) return fail(GYM_E_OOM, "serving: request pool exhausted at admission");
  Slot* sl = new Slot{};
  sl->schur = e->schur;
  sl->mem = mem;
  sl->id = p.id;
  sl->problem = p.req.problem;
  sl->degree = p.req.degree;
  sl->want_x = p.req.want_solution != 0;
  sl->t0 = p.t0;
  sl->op = e;
  sl->n = p.n;
  sl->nb = vec_grid(p.n, s->ctx->ncu);
  sl->bytes = p.slot_bytes;
  sl->sw0 = sl->sw1 = nullptr;
  double* base = (double*)sl->mem;
  double** vecs[10] = {&sl->b, &sl->x, &sl->r1, &sl->r2, &sl->y, &sl->z, &sl->zp, &sl->w, &sl->w1, &sl->w2};
  for (int k = 0; k < 10; ++k) *vecs[k] = base + (size_t)k * p.n;
  double* q = base + 10 * (size_t)p.n;
  sl->pa = q;
  q += (size_t)p.req.nel * p.req.nel * p.req.nel;
  for (int k = 0; k < 2; ++k) {
    sl->pb[k] = q;
    sl->pc[k] = q + sl->nb;
    sl->alfa[k] = q + 2 * sl->nb;
    q += 2 * sl->nb + 1;
  }
  sl->scratch = q;
  sl->sums = q + sl->nb;
  if (sl->schur) {
    sl->sw0 = q + sl->nb + 2;
    sl->sw1 = sl->sw0 + p.np;
  }
  sl->R0[0] = sl->r1, sl->R0[1] = sl->r2, sl->R0[2] = sl->y;
  sl->Z0[0] = sl->z, sl->Z0[1] = sl->zp;
  sl->W0[0] = sl->w, sl->W0[1] = sl->w1, sl->W0[2] = sl->w2;
  sl->tighten = 0;
  sl->par = 0;
  sl->pending = false;
  sl->npa = 0;
  e->refs += 1;
  s->bytes_used += sl->bytes;
  sl->sidx = s->free_sidx.back();
  s->free_sidx.pop_back();
  sl->it = 0;
  int64_t nblk[2];
  gym_op_block_sizes(e->op, nblk);
  if (!p.rhs.empty()) {
    GYM_HIP(hipMemcpyAsync(sl->b, p.rhs.data(), sizeof(double) * p.n, hipMemcpyHostToDevice, s->stream));
    GYM_HIP(hipStreamSynchronize(s->stream));  // the host vector is released below
  } else {
    launch_rhs_normal(sl->b, nblk[0], p.n, p.req.seed, sl->nb, s->stream);
  }
  // init: r1 = r2 = b, z = M^-1 b, beta_1 (y receives v_1, unused)
  MinresVecs<double> V{sl->b, sl->x, sl->r1, sl->r2, sl->z, sl->y, sl->w, sl->w1, sl->w2};
  if (sl->schur) {
    minres_launch_init_vecs<double>(V, p.n, 1, sl->nb, s->stream);
    if (launch_schur_apply<double>(*sl->schur, sl->b, sl->z, 1, sl->nb, s->stream)) {
      s->pool.give((char*)sl->mem, sl->bytes);
      s->bytes_used -= sl->bytes;
      e->refs -= 1;
      s->free_sidx.push_back(sl->sidx);
      delete sl;
      return fail(GYM_E_HIP, "serving: preconditioner launch failed");
    }
    minres_launch_dot2<double>(sl->b, sl->z, nullptr, p.n, 1, sl->nb, sl->scratch, nullptr, s->stream);
    minres_launch_init_state<double>(V, p.n, 1, sl->nb, sl->scratch, s->d_states + 2 * sl->sidx, s->opts.rtol,
                                     s->stream);
  } else {
    minres_launch_init<double>(V, e->op->d_prec, p.n, 1, sl->nb, sl->scratch, s->d_states + 2 * sl->sidx,
                               s->opts.rtol, s->stream);
  }
  s->active.push_back(sl);
  return 0;
}

// One fused MINRES step of every active request.
int step(gym_server* s) {
  const int st = s->stage = (s->stage + 1) % kStages;
  GYM_HIP(hipEventSynchronize(s->ev[st]));
  // first half: operator applies with the fused epilogue, one ragged launch per (problem, degree)
  std::map<std::pair<int, int>, std::vector<Slot*>> groups;
  for (Slot* sl : s->active) groups[{sl->problem, sl->degree}].push_back(sl);
  int off = 0, boff = 0;
  for (auto& g : groups) {
    const auto& list = g.second;
    int prob = 0;
    for (size_t i = 0; i < list.size(); ++i) {
      Slot* sl = list[i];
      OpParams& p = s->plist_h[st][off + i];
      build_op_params(sl->op->op, sl->z, sl->y, p, prob);
      p.fused = 1;
      p.mr = MrStep{s->d_states + 2 * sl->sidx + (sl->it & 1), sl->pa};
    }
    int rc = launch_op_batch(prob, 3, g.first.second, s->plist_h[st] + off, s->bst_h[st] + boff, (int)list.size(),
                             s->plist_d[st] + off, s->bst_d[st] + boff, s->ctx->ncu, s->stream);
    if (rc) return fail(GYM_E_HIP, "serving: batched operator launch failed");
    for (size_t i = 0; i < list.size(); ++i) list[i]->npa = s->bst_h[st][boff + i + 1] - s->bst_h[st][boff + i];
    off += (int)list.size();
    boff += (int)list.size() + 1;
  }
  // second half over all requests
  const int na = (int)s->active.size();
  int nblocks = 0;
  for (int i = 0; i < na; ++i) {
    Slot* sl = s->active[i];
    MrItem& it = s->items_h[st][i];
    it.n = sl->n;
    it.nb = sl->nb;
    it.pad = 0;
    it.v = MrVecs<double>{sl->y, sl->r1, sl->r2, sl->zp, sl->x, sl->w2, sl->w, sl->w1};
    it.dinv = sl->op->op->d_prec;
    MinresState* cur = s->d_states + 2 * sl->sidx + (sl->it & 1);
    MinresState* next = s->d_states + 2 * sl->sidx + ((sl->it + 1) & 1);
    const int pr = sl->par;
    it.io = Step2Io{cur,          next,           sl->pending ? 0 : 1, sl->npa,       sl->nb,
                    sl->pa,       sl->pb[pr],     sl->pc[pr],          sl->alfa[pr],  sl->pb[pr ^ 1],
                    sl->pc[pr ^ 1], sl->alfa[pr ^ 1], sl->schur ? 1 : 0};
    s->ibst_h[st][i] = nblocks;
    nblocks += sl->nb;
  }
  s->ibst_h[st][na] = nblocks;
  GYM_HIP(hipMemcpyAsync(s->items_d[st], s->items_h[st], sizeof(MrItem) * na, hipMemcpyHostToDevice, s->stream));
  GYM_HIP(hipMemcpyAsync(s->ibst_d[st], s->ibst_h[st], sizeof(int) * (na + 1), hipMemcpyHostToDevice, s->stream));
  launch_batch_step2(s->items_d[st], s->ibst_d[st], na, nblocks, s->stream);
  // block-preconditioned requests: z_{k+1} = P^-1 y over zp and the partial
  // sums the second half left out, one ragged batch over all of them (nothing
  // for a request that has converged: its buffers must stay as they were for
  // a resumed recurrence)
  {
    const int maxs = s->opts.max_slots;
    SchurItem* items = s->sitems_h[st];
    int* et = s->stab_h[st];
    int* at[3] = {et + (maxs + 1), et + 2 * (maxs + 1), et + 3 * (maxs + 1)};
    int k = 0;
    et[0] = at[0][0] = at[1][0] = at[2][0] = 0;
    for (Slot* sl : s->active) {
      if (!sl->schur) continue;
      const SchurPrec& P = *sl->schur;
      SchurItem& it = items[k];
      it.ns = P.ns;
      it.np = P.np;
      for (int a = 0; a < 3; ++a) {
        it.m[a] = P.m[a];
        it.fwd[a] = P.fwd64[a];
        it.bwd[a] = P.bwd64[a];
      }
      it.nb = sl->nb;
      it.scale = P.scale;
      it.dsinv = P.dsinv;
      it.lam = P.lam;
      it.y = sl->y;
      it.z = sl->zp;
      it.w0 = sl->sw0;
      it.w1 = sl->sw1;
      it.r2 = sl->r2;
      it.pb = sl->pb[sl->par ^ 1];
      it.pc = sl->pc[sl->par ^ 1];
      it.gate = s->d_states + 2 * sl->sidx + (sl->it & 1);
      et[k + 1] = et[k] + it.nb;
      for (int a = 0; a < 3; ++a) at[a][k + 1] = at[a][k] + schur_axis_blocks(it, a);
      ++k;
    }
    if (k > 0) {
      GYM_HIP(hipMemcpyAsync(s->sitems_d[st], items, sizeof(SchurItem) * k, hipMemcpyHostToDevice, s->stream));
      GYM_HIP(hipMemcpyAsync(s->stab_d[st], et, sizeof(int) * 4 * (maxs + 1), hipMemcpyHostToDevice, s->stream));
      const int* atd[3] = {s->stab_d[st] + (maxs + 1), s->stab_d[st] + 2 * (maxs + 1), s->stab_d[st] + 3 * (maxs + 1)};
      const int na[3] = {at[0][k], at[1][k], at[2][k]};
      launch_schur_batch(s->sitems_d[st], k, s->stab_d[st], et[k], atd, na, s->stream);
    }
  }
  GYM_HIP(hipEventRecord(s->ev[st], s->stream));
  GYM_HIP(hipGetLastError());
  // the same rotation as the single-request driver
  for (Slot* sl : s->active) {
    if (sl->pending) {
      double *w = sl->w, *w1 = sl->w1, *w2 = sl->w2;
      sl->w = w1;
      sl->w1 = w2;
      sl->w2 = w;
    }
    std::swap(sl->z, sl->zp);
    double* r1 = sl->r1;
    sl->r1 = sl->r2;
    sl->r2 = sl->y;
    sl->y = r1;
    sl->pending = true;
    sl->par ^= 1;
    sl->it += 1;
  }
  return 0;
}

// Buffer roles after k working MINRES steps (the host kept rotating while
// the request sat converged on the device, but no kernel touched it).
void roles_from_steps(Slot* sl, int k) {
  sl->r1 = sl->R0[k % 3];
  sl->r2 = sl->R0[(k + 1) % 3];
  sl->y = sl->R0[(k + 2) % 3];
  sl->z = sl->Z0[k & 1];
  sl->zp = sl->Z0[(k + 1) & 1];
  const int kw = k > 0 ? k - 1 : 0;  // the first step does not rotate the w buffers
  sl->w = sl->W0[kw % 3];
  sl->w1 = sl->W0[(kw + 1) % 3];
  sl->w2 = sl->W0[(kw + 2) % 3];
  sl->par = k & 1;
  sl->pending = k > 0;
}

// true relative residual ||b - A x|| / ||b|| in FP64 (y is scratch between
// steps)
int true_relres(gym_server* s, Slot* sl, double* rel) {
  if (int rc = launch_op_apply(sl->op->op, GYM_F64, 1, sl->x, sl->y, s->stream)) return rc;
  launch_norm2(sl->y, sl->b, sl->n, 1, sl->nb, 1, sl->scratch, sl->sums, s->stream);
  launch_norm2(sl->b, nullptr, sl->n, 1, sl->nb, 0, sl->scratch, sl->sums + 1, s->stream);
  double h[2];
  GYM_HIP(hipMemcpyAsync(h, sl->sums, sizeof(h), hipMemcpyDeviceToHost, s->stream));
  GYM_HIP(hipStreamSynchronize(s->stream));
  double bn = std::sqrt(h[1]);
  *rel = bn > 0 ? std::sqrt(h[0]) / bn : std::sqrt(h[0]);
  return 0;
}

int retire(gym_server* s, Slot* sl, const MinresState& ms, double rel) {
  Done d;
  if (sl->want_x) {
    d.x.resize(sl->n);
    GYM_HIP(hipMemcpyAsync(d.x.data(), sl->x, sizeof(double) * sl->n, hipMemcpyDeviceToHost, s->stream));
    GYM_HIP(hipStreamSynchronize(s->stream));
  }
  d.res.rel_res = rel;
  d.res.iters = ms.itn;
  d.res.ndofs = sl->n;
  d.res.status = ms.flag < 0 ? GYM_E_BREAKDOWN : (d.res.rel_res <= s->opts.rtol ? GYM_OK : GYM_W_NOT_CONVERGED);
  d.res.latency_s = std::chrono::duration<double>(Clock::now() - sl->t0).count();
  s->pool.give((char*)sl->mem, sl->bytes);
  s->bytes_used -= sl->bytes;
  sl->op->refs -= 1;
  s->free_sidx.push_back(sl->sidx);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->pending.erase(sl->id);
    s->done[sl->id] = std::move(d);
  }
  s->cv.notify_all();
  return 0;
}

int check_and_retire(gym_server* s) {
  if (s->active.empty()) return 0;
  const int maxs = s->opts.max_slots;
  GYM_HIP(hipMemcpyAsync(s->h_states, s->d_states, sizeof(MinresState) * 2 * maxs, hipMemcpyDeviceToHost, s->stream));
  GYM_HIP(hipStreamSynchronize(s->stream));
  std::vector<Slot*> keep;
  for (Slot* sl : s->active) {
    MinresState ms = s->h_states[2 * sl->sidx + (sl->it & 1)];
    if (ms.done || sl->it >= s->opts.maxit) {
      if (ms.done) {
        // converged when step itn was closed, in working step itn + 1
        roles_from_steps(sl, ms.itn + 1);
      } else if (sl->pending) {
        // iteration cap: complete the pending step so that x is its iterate
        MinresState* cur = s->d_states + 2 * sl->sidx + (sl->it & 1);
        MinresState* next = s->d_states + 2 * sl->sidx + ((sl->it + 1) & 1);
        minres_launch_finish<double>(sl->x, sl->zp, sl->w2, sl->w, sl->w1, sl->n, 1, sl->nb, cur, next,
                                     sl->pb[sl->par], sl->alfa[sl->par], s->stream);
        GYM_HIP(hipMemcpyAsync(&ms, next, sizeof(MinresState), hipMemcpyDeviceToHost, s->stream));
        GYM_HIP(hipStreamSynchronize(s->stream));
      }
      double rel = 0;
      if (int rc = true_relres(s, sl, &rel)) return rc;
      if (ms.done && rel > s->opts.rtol && ms.flag >= 0 && sl->it < s->opts.maxit && sl->tighten < 6) {
        // the preconditioned estimate was optimistic: tighten and resume
        // the same recurrence (the pending step is closed next)
        sl->tighten += 1;
        ms.tol *= 0.1;
        ms.done = 0;
        ms.flag = 0;
        MinresState pair[2] = {ms, ms};
        GYM_HIP(hipMemcpyAsync(s->d_states + 2 * sl->sidx, pair, sizeof(pair), hipMemcpyHostToDevice, s->stream));
        GYM_HIP(hipStreamSynchronize(s->stream));
        keep.push_back(sl);
        continue;
      }
      if (int rc = retire(s, sl, ms, rel)) return rc;
      delete sl;
    } else {
      keep.push_back(sl);
    }
  }
  s->active.swap(keep);
  return 0;
}

void loop(gym_server* s) {
  if (hipSetDevice(s->ctx->device) != hipSuccess) {
    record_fatal(s, GYM_E_HIP);
    return;
  }
  int steps = 0;
  for (;;) {
    // admission
    for (;;) {
      Pending p;
      {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->queue.empty() || (int)s->active.size() >= s->opts.max_slots) break;
        Pending& f = s->queue.front();
        size_t need = f.bytes;
        const size_t block = f.slot_bytes;
        lk.unlock();
        if (s->bytes_used + need > (size_t)s->opts.mem_budget) evict_ops(s, need);
        lk.lock();
        if (s->bytes_used + need > (size_t)s->opts.mem_budget || !s->pool.fits(block)) break;
        p = std::move(s->queue.front());
        s->queue.pop_front();
      }
      if (int rc = admit(s, p)) {
        std::lock_guard<std::mutex> lk(s->mu);
        Done d;
        d.res.status = rc;
        s->pending.erase(p.id);
        s->done[p.id] = std::move(d);
        s->cv.notify_all();
      }
    }
    if (s->active.empty()) {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stopping && s->queue.empty()) break;
      s->cv.wait_for(lk, std::chrono::milliseconds(1));
      continue;
    }
    if (step(s)) {
      record_fatal(s, GYM_E_HIP);
      return;
    }
    if (++steps % kCheckEvery == 0) {
      if (check_and_retire(s)) {
        record_fatal(s, GYM_E_HIP);
        return;
      }
    }
  }
}

}  // namespace

extern "C" {

int gym_serve_start(const gym_serve_opts* opts, gym_server** out) {
  if (!opts || !out) return fail(GYM_E_ARG, "NULL argument");
  if (opts->max_slots < 1 || opts->max_slots > 4096 || opts->mem_budget <= 0 || opts->maxit < 1 || !(opts->rtol > 0))
    return fail(GYM_E_ARG, "bad serving options");
  if (opts->precond != GYM_PRECOND_JACOBI && opts->precond != GYM_PRECOND_SCHUR)
    return fail(GYM_E_ARG, "serving preconditioner must be GYM_PRECOND_JACOBI or GYM_PRECOND_SCHUR");
  gym_server* s = new gym_server;
  s->opts = *opts;
  if (int rc = gym_create(&s->ctx, opts->device)) {
    delete s;
    return rc;
  }
  GYM_HIP(hipStreamCreate(&s->stream));
  // the request pool: one allocation for the server's lifetime
  if (hipMalloc(&s->pool_mem, (size_t)opts->mem_budget) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamDestroy(s->stream);
    gym_destroy(s->ctx);
    delete s;
    return fail(GYM_E_OOM, "serving: cannot reserve the memory budget on the device");
  }
  s->pool.reset((char*)s->pool_mem, (size_t)opts->mem_budget);
  const int maxs = opts->max_slots;
  GYM_HIP(hipMalloc(&s->d_states, sizeof(MinresState) * 2 * maxs));
  GYM_HIP(hipHostMalloc((void**)&s->h_states, sizeof(MinresState) * 2 * maxs, hipHostMallocDefault));
  for (int i = maxs - 1; i >= 0; --i) s->free_sidx.push_back(i);
  for (int k = 0; k < kStages; ++k) {
    GYM_HIP(hipHostMalloc((void**)&s->plist_h[k], sizeof(OpParams) * maxs, hipHostMallocDefault));
    GYM_HIP(hipMalloc(&s->plist_d[k], sizeof(OpParams) * maxs));
    GYM_HIP(hipHostMalloc((void**)&s->bst_h[k], sizeof(int) * (maxs + kMaxGroups + 1), hipHostMallocDefault));
    GYM_HIP(hipMalloc(&s->bst_d[k], sizeof(int) * (maxs + kMaxGroups + 1)));
    GYM_HIP(hipHostMalloc((void**)&s->items_h[k], sizeof(MrItem) * maxs, hipHostMallocDefault));
    GYM_HIP(hipMalloc(&s->items_d[k], sizeof(MrItem) * maxs));
    GYM_HIP(hipHostMalloc((void**)&s->ibst_h[k], sizeof(int) * (maxs + 1), hipHostMallocDefault));
    GYM_HIP(hipMalloc(&s->ibst_d[k], sizeof(int) * (maxs + 1)));
    GYM_HIP(hipHostMalloc((void**)&s->sitems_h[k], sizeof(SchurItem) * maxs, hipHostMallocDefault));
    GYM_HIP(hipMalloc(&s->sitems_d[k], sizeof(SchurItem) * maxs));
    GYM_HIP(hipHostMalloc((void**)&s->stab_h[k], sizeof(int) * 4 * (maxs + 1), hipHostMallocDefault));
    GYM_HIP(hipMalloc(&s->stab_d[k], sizeof(int) * 4 * (maxs + 1)));
    GYM_HIP(hipEventCreate(&s->ev[k]));
    GYM_HIP(hipEventRecord(s->ev[k], s->stream));
  }
  s->th = std::thread(loop, s);
  *out = s;
  return GYM_OK;
}

int gym_serve_submit(gym_server* s, const gym_request* req, uint64_t* id) {
  if (!s || !req || !id) return fail(GYM_E_ARG, "NULL argument");
  if ((req->problem != GYM_MIXED_POISSON && req->problem != GYM_HODGE1) || req->nel < 1 || req->nel > 1024 ||
      req->degree < 1 || req->degree > kMaxR)
    return fail(GYM_E_ARG, "bad request");
  if (s->opts.precond == GYM_PRECOND_SCHUR && req->problem != GYM_MIXED_POISSON)
    return fail(GYM_E_UNSUPPORTED, "the block preconditioner serves mixed Poisson requests only");
  Pending p;
  p.req = *req;
  p.n = request_ndofs(*req);
  p.bytes = request_bytes(p.n, req->nel, s->ctx->ncu);
  // with the block preconditioner: two cell-block work vectors of its own
  p.np = (int64_t)req->degree * req->nel * (int64_t)req->degree * req->nel * (int64_t)req->degree * req->nel;
  const size_t extra = s->opts.precond == GYM_PRECOND_SCHUR ? 2 * (size_t)p.np : 0;
  p.slot_bytes = sizeof(double) * (slot_doubles(p.n, req->nel, vec_grid(p.n, s->ctx->ncu)) + extra);
  p.bytes += sizeof(double) * extra;
  if (p.bytes > (size_t)s->opts.mem_budget) return fail(GYM_E_OOM, "request exceeds the server's memory budget");
  if (req->rhs) p.rhs.assign(req->rhs, req->rhs + p.n);
  p.req.rhs = nullptr;
  p.t0 = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(GYM_E_ARG, "server is stopping");
    p.id = s->next_id++;
    s->pending[p.id] = 1;
    *id = p.id;
    s->queue.push_back(std::move(p));
  }
  s->cv.notify_all();
  return GYM_OK;
}

int gym_serve_poll(gym_server* s, uint64_t id, gym_result* res, double* x_host) {
  if (!s || !res) return fail(GYM_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fatal) return fail(s->fatal, "serving loop stopped: " + s->fatal_msg);
  auto it = s->done.find(id);
  if (it == s->done.end()) {
    if (s->pending.count(id)) {
      res->status = 2;
      return 2;
    }
    return fail(GYM_E_ARG, "unknown request id");
  }
  *res = it->second.res;
  if (x_host && !it->second.x.empty()) std::copy(it->second.x.begin(), it->second.x.end(), x_host);
  s->done.erase(it);
  return 0;
}

int gym_serve_stop(gym_server* s) {
  if (!s) return GYM_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  int rc = s->fatal;
  for (Slot* sl : s->active) delete sl;
  for (auto& kv : s->ops) {
    gym_op_destroy(kv.second->op);
    gym_mesh_destroy(kv.second->mesh);
    delete kv.second;
  }
  for (int k = 0; k < kStages; ++k) {
    (void)hipHostFree(s->plist_h[k]);
    (void)hipFree(s->plist_d[k]);
    (void)hipHostFree(s->bst_h[k]);
    (void)hipFree(s->bst_d[k]);
    (void)hipHostFree(s->items_h[k]);
    (void)hipFree(s->items_d[k]);
    (void)hipHostFree(s->ibst_h[k]);
    (void)hipFree(s->ibst_d[k]);
    (void)hipHostFree(s->sitems_h[k]);
    (void)hipFree(s->sitems_d[k]);
    (void)hipHostFree(s->stab_h[k]);
    (void)hipFree(s->stab_d[k]);
    (void)hipEventDestroy(s->ev[k]);
  }
  (void)hipFree(s->d_states);
  (void)hipFree(s->pool_mem);
  (void)hipHostFree(s->h_states);
  (void)hipStreamDestroy(s->stream);
  gym_destroy(s->ctx);
  delete s;
  return rc ? fail(rc, "serving loop had stopped on an error") : GYM_OK;
}

}  // extern "C"
