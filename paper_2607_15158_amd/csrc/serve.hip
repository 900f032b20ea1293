// Continuous batching of environment solves on one GPU.
//
// A server owns one device arena, allocated once, and a fixed number of
// slots, each with its own HIP stream.  Requests (a site tensor, a
// configuration, optional start blocks and a bond operator) wait in a queue
// and are admitted while a slot is free and their footprint -- the
// context workspace of ctm_workspace_bytes plus their staged inputs -- fits
// into the free part of the arena (first fit; a request that does not fit
// does not hold back smaller ones behind it).  Every running request is one
// context on its slot's stream with C, T, X and Y resident in its
// workspace; each pump completes the moves that have finished, launches the
// next move of every request that is still iterating, retires requests that
// reached delta < tol (at the full environment dimension) or their move
// budget, and admits new ones.  SI moves replay a captured HIP graph per
// request, or, for requests up to a size set by ctm_server_batching, move
// together through ctm_move_batch_async (grouped launches over all of them).  Moves of different requests therefore overlap on the device,
// and a result does not depend on what else runs:
// each request executes exactly the kernels, launch shapes and reduction
// orders of a solo ctm_converge.

#include "../../include/ctm.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request {
  ctm_config cfg{};
  std::vector<double> site, boundary, X0, Yt0, op;
  double tol = 0.0;
  int max_moves = 0;
  ctm_result res{};
  ctm_ctx* ctx = nullptr;
  int slot = -1;
  size_t off = 0, bytes = 0, ws_bytes = 0;
  std::string err;
};

}  // namespace

struct ctm_server {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  std::map<size_t, size_t> free_blocks;   // offset -> size
  std::vector<hipStream_t> streams;
  std::vector<int> slot_req;              // request id per slot, -1 if free
  std::vector<Request> reqs;
  std::chrono::steady_clock::time_point t0;
  std::string err;
  // batched moves: requests with chi * Dl <= batch_max_n whose next move is
  // an SI move move together through ctm_move_batch_async (0: every request
  // moves on its own slot stream)
  int batch_max_n = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t roff = it->first + bytes;
        free_blocks.erase(it);
        if (rest) free_blocks[roff] = rest;
        return true;
      }
    }
    return false;
  }

  void release(size_t off, size_t bytes) {
    auto it = free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_blocks.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blocks.erase(nx);
    }
    if (it != free_blocks.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blocks.erase(it);
      }
    }
  }
};

namespace {

int dims(const ctm_config& c, size_t* nsite, size_t* Dl, size_t* nk) {
  const size_t D = c.D;
  *Dl = c.d > 0 ? D * D : D;
  *nsite = c.d > 0 ? (size_t)c.d * D * D * D * D : (*Dl) * (*Dl) * (*Dl) * (*Dl);
  const size_t N = (size_t)c.chi * (*Dl);
  const size_t k = std::min<size_t>((size_t)c.chi + c.p, N);
  *nk = N * k;
  return 0;
}

// Device layout of a request's block: workspace, site, boundary, X0, Yt0.
struct Staging {
  size_t ws, site, boundary, iso, total;
};

Staging staging(const Request& r) {
  size_t nsite, Dl, nk;
  dims(r.cfg, &nsite, &Dl, &nk);
  Staging s;
  s.ws = align_up(r.ws_bytes);
  s.site = align_up(nsite * 8);
  s.boundary = r.boundary.empty() ? 0 : align_up(Dl * 8);
  s.iso = r.X0.empty() ? 0 : align_up(4 * nk * 8);
  s.total = s.ws + s.site + s.boundary + 2 * s.iso;
  return s;
}

void retire(ctm_server* s, int id, int state) {
  Request& r = s->reqs[id];
  if (r.ctx) {
    ctm_destroy(r.ctx);
    r.ctx = nullptr;
  }
  if (r.bytes) s->release(r.off, r.bytes);
  r.bytes = 0;
  if (r.slot >= 0) s->slot_req[r.slot] = -1;
  r.slot = -1;
  r.res.state = state;
  r.res.t_done = s->now();
  // inputs are no longer needed
  r.site.clear();
  r.boundary.clear();
  r.X0.clear();
  r.Yt0.clear();
}

void fail_request(ctm_server* s, int id, const char* what) {
  Request& r = s->reqs[id];
  r.err = std::string(what) + ": " + ctm_last_error(r.ctx);
  retire(s, id, 3);
}

// Admits request id into slot; returns false (and leaves it queued) if its
// footprint does not fit.
bool admit(ctm_server* s, int id, int slot) {
  Request& r = s->reqs[id];
  const Staging st = staging(r);
  size_t off;
  if (!s->alloc(st.total, &off)) return false;
  r.off = off;
  r.bytes = st.total;
  r.slot = slot;
  s->slot_req[slot] = id;
  r.res.state = 1;
  r.res.t_admit = s->now();
  r.res.bytes = st.total;
  hipStream_t stream = s->streams[slot];
  char* base = s->arena + off;
  double* site = (double*)(base + st.ws);
  double* bnd = st.boundary ? (double*)(base + st.ws + st.site) : nullptr;
  double* X0 = st.iso ? (double*)(base + st.ws + st.site + st.boundary) : nullptr;
  double* Y0 = st.iso ? (double*)(base + st.ws + st.site + st.boundary + st.iso) : nullptr;
  bool ok = hipMemcpyAsync(site, r.site.data(), r.site.size() * 8, hipMemcpyHostToDevice, stream) ==
            hipSuccess;
  if (ok && bnd)
    ok = hipMemcpyAsync(bnd, r.boundary.data(), r.boundary.size() * 8, hipMemcpyHostToDevice,
                        stream) == hipSuccess;
  if (ok && X0)
    ok = hipMemcpyAsync(X0, r.X0.data(), r.X0.size() * 8, hipMemcpyHostToDevice, stream) ==
             hipSuccess &&
         hipMemcpyAsync(Y0, r.Yt0.data(), r.Yt0.size() * 8, hipMemcpyHostToDevice, stream) ==
             hipSuccess;
  if (!ok) {
    r.err = "copy of the request inputs failed";
    retire(s, id, 3);
    return true;
  }
  if (ctm_init(&r.ctx, &r.cfg, site, bnd, base, st.ws, stream) != CTM_OK) {
    r.err = std::string("ctm_init: ") + ctm_last_error(nullptr);
    retire(s, id, 3);
    return true;
  }
  // SI moves replay captured graphs (the slot stream is not the default one)
  if (ctm_use_graphs(r.ctx, 1) != CTM_OK) {
    fail_request(s, id, "ctm_use_graphs");
    return true;
  }
  if (X0 && ctm_set_isometries(r.ctx, X0, Y0) != CTM_OK) {
    fail_request(s, id, "ctm_set_isometries");
    return true;
  }
  if (r.max_moves == 0) {
    retire(s, id, 2);
    return true;
  }
  if (ctm_move_async(r.ctx) != CTM_OK) fail_request(s, id, "ctm_move_async");
  return true;
}

void finish(ctm_server* s, int id) {
  Request& r = s->reqs[id];
  double out[8];
  if (ctm_observable(r.ctx, CTM_OBS_NORM, nullptr, out) != CTM_OK) {
    fail_request(s, id, "norm");
    return;
  }
  r.res.kappa = out[0];
  if (!r.op.empty()) {
    if (ctm_observable(r.ctx, CTM_OBS_BOND_H, r.op.data(), out) != CTM_OK) {
      fail_request(s, id, "horizontal bond");
      return;
    }
    r.res.bond_h = out[0];
    if (ctm_observable(r.ctx, CTM_OBS_BOND_V, r.op.data(), out) != CTM_OK) {
      fail_request(s, id, "vertical bond");
      return;
    }
    r.res.bond_v = out[0];
  }
  retire(s, id, 2);
}

}  // namespace

extern "C" {

ctm_status ctm_server_create(ctm_server** out, size_t arena_bytes, int max_slots) {
  if (!out || arena_bytes == 0 || max_slots < 1 || max_slots > 64) return CTM_E_ARG;
  *out = nullptr;
  ctm_server* s = new ctm_server();
  s->arena_bytes = arena_bytes / kAlign * kAlign;
  if (hipMalloc((void**)&s->arena, s->arena_bytes) != hipSuccess) {
    delete s;
    return CTM_E_NOMEM;
  }
  s->free_blocks[0] = s->arena_bytes;
  s->streams.resize(max_slots, nullptr);
  for (auto& st : s->streams) {
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      ctm_server_destroy(s);
      return CTM_E_DEVICE;
    }
  }
  s->slot_req.assign(max_slots, -1);
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return CTM_OK;
}

void ctm_server_destroy(ctm_server* s) {
  if (!s) return;
  for (size_t i = 0; i < s->reqs.size(); ++i)
    if (s->reqs[i].ctx) retire(s, (int)i, 3);
  for (auto st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
}

ctm_status ctm_server_submit(ctm_server* s, const ctm_config* cfg, const double* site_host,
                             const double* boundary_host, const double* X0_host,
                             const double* Yt0_host, const double* op_host, double tol,
                             int max_moves, int* id) {
  if (!s || !cfg || !site_host || !id || max_moves < 0 || (X0_host == nullptr) != (Yt0_host == nullptr))
    return CTM_E_ARG;
  size_t wsb = 0;
  const ctm_status v = ctm_workspace_bytes(cfg, &wsb);
  if (v != CTM_OK) return v;
  if (cfg->d == 0 && !boundary_host) return CTM_E_ARG;
  Request r;
  r.cfg = *cfg;
  r.ws_bytes = wsb;
  size_t nsite, Dl, nk;
  dims(*cfg, &nsite, &Dl, &nk);
  r.site.assign(site_host, site_host + nsite);
  if (boundary_host) r.boundary.assign(boundary_host, boundary_host + Dl);
  if (X0_host) {
    r.X0.assign(X0_host, X0_host + 4 * nk);
    r.Yt0.assign(Yt0_host, Yt0_host + 4 * nk);
  }
  if (op_host && cfg->d > 0) {
    const size_t d2 = (size_t)cfg->d * cfg->d;
    r.op.assign(op_host, op_host + d2 * d2);
  }
  r.tol = tol;
  r.max_moves = max_moves;
  if (staging(r).total > s->arena_bytes) return CTM_E_NOMEM;
  r.res.state = 0;
  r.res.t_submit = s->now();
  s->reqs.push_back(std::move(r));
  *id = (int)s->reqs.size() - 1;
  return CTM_OK;
}

ctm_status ctm_server_pump(ctm_server* s, int* n_running, int* n_queued) {
  if (!s) return CTM_E_ARG;
  // 1. completed moves: retire, or queue the next move
  std::vector<int> batch;
  for (size_t slot = 0; slot < s->slot_req.size(); ++slot) {
    const int id = s->slot_req[slot];
    if (id < 0) continue;
    Request& r = s->reqs[id];
    int done = 0;
    ctm_move_info info{};
    if (ctm_move_poll(r.ctx, &done, &info) != CTM_OK) {
      fail_request(s, id, "move");
      continue;
    }
    if (!done) continue;
    r.res.moves += 1;
    r.res.delta = info.delta;
    const bool conv = (info.mode != 0) && info.chi_env == r.cfg.chi && info.delta < r.tol;
    if (conv || r.res.moves >= r.max_moves) {
      r.res.converged = conv ? 1 : 0;
      finish(s, id);
      continue;
    }
    size_t nsite, Dl, nk;
    dims(r.cfg, &nsite, &Dl, &nk);
    const bool si_next = info.chi_env == r.cfg.chi && r.cfg.proj == CTM_PROJ_SI &&
                         r.cfg.prec == CTM_PREC_F64 && r.cfg.sym == CTM_SYM_NONE;
    if (s->batch_max_n > 0 && si_next && (long)r.cfg.chi * (long)Dl <= s->batch_max_n)
      batch.push_back(id);
    else if (ctm_move_async(r.ctx) != CTM_OK)
      fail_request(s, id, "ctm_move_async");
  }
  // the next moves of the batched requests: one grouped launch sequence
  if (!batch.empty()) {
    std::vector<ctm_ctx*> cs;
    for (int id : batch) cs.push_back(s->reqs[id].ctx);
    if (ctm_move_batch_async(cs.data(), (int)cs.size()) != CTM_OK)
      for (int id : batch) fail_request(s, id, "ctm_move_batch_async");
  }
  // 2. admission, in submission order, first fit
  for (size_t id = 0; id < s->reqs.size(); ++id) {
    if (s->reqs[id].res.state != 0) continue;
    int slot = -1;
    for (size_t k = 0; k < s->slot_req.size(); ++k)
      if (s->slot_req[k] < 0) {
        slot = (int)k;
        break;
      }
    if (slot < 0) break;
    admit(s, (int)id, slot);
  }
  int run = 0, queued = 0;
  for (const auto& r : s->reqs) {
    run += r.res.state == 1;
    queued += r.res.state == 0;
  }
  if (n_running) *n_running = run;
  if (n_queued) *n_queued = queued;
  return CTM_OK;
}

ctm_status ctm_server_batching(ctm_server* s, int max_n) {
  if (!s || max_n < 0) return CTM_E_ARG;
  s->batch_max_n = max_n;
  return CTM_OK;
}

ctm_status ctm_server_result(const ctm_server* s, int id, ctm_result* out) {
  if (!s || !out || id < 0 || id >= (int)s->reqs.size()) return CTM_E_ARG;
  *out = s->reqs[id].res;
  return CTM_OK;
}

const char* ctm_server_error(const ctm_server* s, int id) {
  if (!s || id < 0 || id >= (int)s->reqs.size()) return "";
  return s->reqs[id].err.c_str();
}

double ctm_server_clock(const ctm_server* s) { return s ? s->now() : 0.0; }

}  // extern "C"
