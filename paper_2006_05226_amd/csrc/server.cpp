// Serving loop: continuous batching of MLCC excitation solves of uneven size
// on one GPU.
//
// * mlcc_submit (any host thread) validates the request, reserves its host
//   bytes against the host budget, copies its inputs to host memory owned by
//   the request and queues it with a ticket.
// * max_slots execution lanes, each with its own HIP stream (default priority)
//   and its own scratch, run admitted requests concurrently, so the kernels of
//   requests of different sizes overlap on the device.  A lane takes the
//   first queued request whose HBM footprint estimate fits in what the budget
//   has left (FIFO with backfill, admission.h); the host copy of the inputs
//   is dropped once the problem holds them on the device, and memory and the
//   slot are returned when the request finishes and waiting requests are
//   admitted at once.
// * Each request runs its ground state, then the Davidson solve for its roots;
//   the result and the submit / admit / done times go to the ticket table that
//   mlcc_poll reads.  The kernels and reductions are deterministic, so a
//   request gives the same result alone and in a mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <unistd.h>

#include "admission.h"
#include "drivers.h"

namespace mlcc {
namespace {

struct Request {
  uint64_t ticket = 0;
  mlcc_problem_desc desc{};
  std::vector<double> L, eps, fock;  // owned copies (L empty for synthetic inputs)
  int32_t n_roots = 0;
  mlcc_solver_opts gs{}, es{};
  uint64_t footprint = 0;
  uint64_t host_bytes = 0;  // of the copies above, counted against the host budget
  bool done = false;
  mlcc_result res{};
};

struct Lane {
  Exec ex;
  Alloc al;  // the lane's stream-ordered cache over the context's allocator
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace mlcc

using namespace mlcc;

struct mlcc_server {
  mlcc_context *ctx = nullptr;
  int max_slots = 8;
  std::mutex mu;
  std::condition_variable cv;
  std::unique_ptr<Admission<Request>> adm;  // under mu
  std::unordered_map<uint64_t, Request *> table;
  uint64_t next_ticket = 1;
  std::vector<std::unique_ptr<Lane>> lanes;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  void work(Lane *lane);
};

namespace {
// Device bytes of a request's solve peak (L, L~, packed blocks, the
// ground-state u that the Jacobian reads, the pair blocks of the MLCC2
// doubles, the per-vector scratch of a Jacobian batch, the Davidson subspace
// and the DIIS history) before the packed BF16 planes of its large products;
// *setup_out receives the set-up peak (L, plus its FP64 staging copy in FP32
// mode).  0 for invalid input.
// *planes_out receives the packed BF16 planes a split- or plain-BF16 request
// may hold at once (0 for the other tiers and without doubles): those of its
// largest products, the doubles-to-singles products of a pair block or of
// the full doubles (R rows of pairs, b trial vectors, J Cholesky vectors):
// 2 planes x 2 bytes x (1 + b) R x max(J + 1, R), rows and reduction padded,
// at most the engine's cap.  A lane runs the request with this cap, so a
// product whose planes need more runs unpacked.
double solve_bytes(const mlcc_problem_desc *d, int32_t n_roots, const mlcc_solver_opts *es,
                   double *setup_out, double *planes_out);

uint64_t planes_share(const mlcc_problem_desc *d, int32_t n_roots, const mlcc_solver_opts *es) {
  double setup = 0.0, planes = 0.0;
  solve_bytes(d, n_roots, es, &setup, &planes);
  return (uint64_t)planes;
}
}  // namespace

// Device bytes one request needs at its peak, with a 15% margin: the larger
// of the set-up peak and the solve peak (solve_bytes plus the packed planes
// of planes_share), plus the lane's split-K partial sums (at most ~67 MB:
// resident blocks x compute units x the largest FP64 tile) and reduction
// buffers.
extern "C" uint64_t mlcc_request_footprint(const mlcc_problem_desc *d, int32_t n_roots,
                                           const mlcc_solver_opts *es) {
  if (!d || n_roots < 1) return 0;
  double setup = 0.0, planes = 0.0;
  const double run = solve_bytes(d, n_roots, es, &setup, &planes) + planes;
  return (uint64_t)(std::max(setup, run) * 1.15) + (160ull << 20);
}

namespace {
double solve_bytes(const mlcc_problem_desc *d, int32_t n_roots, const mlcc_solver_opts *es,
                   double *setup_out, double *planes_out) {
  *setup_out = *planes_out = 0.0;
  if (!d || n_roots < 1) return 0.0;
  const double O = d->n_occ, V = d->n_vir, J = d->n_chol, n = O + V;
  const bool dbl = d->model != MLCC_CCS && d->n_occ_act > 0 && d->n_vir_act > 0;
  const double o = dbl ? d->n_occ_act : 0.0, v = dbl ? d->n_vir_act : 0.0;
  const double M = o * v, MM = M * M;
  const double ts = d->precision == MLCC_FP64 ? 8.0 : 4.0;
  const double nL = J * n * n, n1 = O * V;
  const bool mlcc2 = d->model == MLCC_MLCC2;
  const bool ccsd = d->model == MLCC_MLCCSD || d->model == MLCC_MLCCSD3;
  // CCSD space of the ladder integrals (three-level MLCCSD: a prefix)
  const double vt = d->model == MLCC_MLCCSD3 ? std::min<double>(d->n_vir_ccsd, v) : v;
  const bool eff = es && es->effective && mlcc2;
  const double dim = n1 + ((dbl && !eff) ? MM : 0.0);
  // trial vectors per Jacobian batch (the rule of the transformation)
  const double per_v = ts * (J * V * O + 2.0 * J * M + J * o * O);
  double bmax = std::floor(48e9 / per_v);
  if (dbl && !eff) bmax = std::min(bmax, std::floor(48e9 / (MM * (16.0 + ts))));
  bmax = std::max(1.0, std::min(8.0, bmax));
  const double b = std::min((double)n_roots + 2.0, bmax);
  const double setup = nL * ts + (ts == 4.0 ? nL * 8.0 : 0.0) + 6.0 * n * n * 8.0;
  double run = 2.0 * nL * ts;                 // L and L~
  run += 8.0 * n * n * 8.0;                   // h, h~, F~, Fock and scratch
  run += 5.0 * (J + 1.0) * M * ts;            // packed L_ai (two orders), L~_ai, Z, dot scratch
  run += J * O * O * ts;                      // L~_oo transposed
  run += b * (per_v + 3.0 * n1 * ts);         // transform batch: W, dL~, Zc, P, trial singles
  // packed planes of a product: 2 planes x 2 bytes per element of a shared
  // operand (ra rows) and z batched ones (rb rows), reduction k
  auto plane_bytes = [](double ra, double rb, double k, double z) {
    auto up = [](double x, double m) { return std::ceil(x / m) * m; };
    return 4.0 * up(k, 64.0) * (up(ra, 256.0) + z * up(rb, 256.0));
  };
  double planes = 0.0;
  if (mlcc2 && dbl) {
    run += MM * ts;                           // ground-state u kept for the Jacobian
    const int nz = eff ? (int)b : 1;
    const double R = std::min((double)mlcc::pair_block_occ((int)o, (int)v, nz, (int)ts), o) * v;
    run += nz * R * R * (16.0 + 2.0 * ts);    // pair blocks of the doubles
    if (!eff) run += MM * b * (8.0 + ts);     // G and u(c2) of full-space batches
    // ground state: g~ and Z of single pair blocks; effective transformation:
    // the same for b vectors; full space: G of the batch
    const double R1 = std::min((double)mlcc::pair_block_occ((int)o, (int)v, 1, (int)ts), o) * v;
    planes = std::max(plane_bytes(R1, R1, J, 1.0), plane_bytes(J + 1.0, R1, R1, 1.0));
    if (eff) planes = std::max({planes, plane_bytes(R, R, J, b), plane_bytes(J + 1.0, R, R, b)});
    else planes = std::max(planes, plane_bytes(M, b * M, J, 1.0));
  }
  if (ccsd && dbl) {
    planes = std::max(plane_bytes(M, M, J, 1.0), plane_bytes(M, b * M, J, 1.0));
    run += MM * (8.0 * 2 + ts * 4) + MM * b * (ts + 8.0);  // t2, Omega_2, u, copies; G, u(c2)
    run += (vt * v * vt * v + O * v * vt * v + O * o * M) * ts + 16.0 * MM * ts;  // integral blocks
  }
  const double space = es && es->max_subspace > 0 ? es->max_subspace : 20.0 * n_roots;
  run += dim * 8.0 * (2.0 * space + 3.0 * (n_roots + 2));  // Davidson
  run += 2.0 * 8.0 * (n1 + (ccsd ? MM : 0.0)) * 8;         // DIIS
  *setup_out = setup;
  if (d->precision == MLCC_BF16X3 || d->precision == MLCC_BF16)
    *planes_out = std::min((double)mlcc::kPlaneBytesMax, planes);
  return run;
}
}  // namespace

void mlcc_server::work(Lane *lane) {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    Request *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        if (adm->stopped()) return;
        r = adm->admit();
        if (r) break;
        cv.wait(lk);
      }
      r->res.t_admit = now_s(t0);
    }
    bool host_held = true;
    auto drop_host = [&]() {
      if (!host_held) return;
      r->L.clear();
      r->L.shrink_to_fit();
      r->fock.clear();
      r->fock.shrink_to_fit();
      std::lock_guard<std::mutex> lk(mu);
      adm->drop_host(r->host_bytes);
      host_held = false;
    };
    mlcc_status st = MLCC_OK;
    mlcc_result &out = r->res;
    out.n_roots = r->n_roots;
    try {
      mlcc_problem_desc d = r->desc;
      d.flags &= ~MLCC_INPUT_ON_DEVICE;  // the inputs are the request's host copies now
      if (!(d.flags & MLCC_SYNTH_L)) d.L = r->L.data();
      d.eps = r->eps.data();
      d.fock = r->fock.empty() ? nullptr : r->fock.data();
      lane->ex.planes_cap = planes_share(&d, r->n_roots, &r->es);
      std::unique_ptr<mlcc_problem> P(problem_new(ctx, &lane->ex, &d));
      drop_host();  // the problem holds its own device copies now
      mlcc_info gi{};
      mlcc_status gs = ground_state(*P, r->gs, gi);
      out.e_corr = gi.energy;
      out.gs_iterations = gi.iterations;
      std::vector<double> w(r->n_roots, 0.0);
      mlcc_info ei{};
      mlcc_status es = mlcc_davidson_solve(P.get(), r->n_roots, &r->es, w.data(), nullptr, &ei);
      out.es_iterations = ei.iterations;
      for (int i = 0; i < r->n_roots && i < 16; ++i) out.omega[i] = w[i];
      st = gs != MLCC_OK ? gs : es;
      P.reset();
      MLCC_HIP(hipStreamSynchronize(lane->ex.stream));
    } catch (const Error &e) {
      st = e.code;
    } catch (...) {
      st = MLCC_E_DEVICE;
    }
    // the lane's split and reduction scratch go back with the request's
    // footprint; with the stream idle, its cached blocks serve every lane
    (void)hipStreamSynchronize(lane->ex.stream);
    lane->ex.work.release();
    lane->ex.red.release();
    lane->ex.planes.release();
    lane->al.quiesce();
    drop_host();
    {
      std::lock_guard<std::mutex> lk(mu);
      adm->release(r->footprint);
      out.status = st;
      out.t_done = now_s(t0);
      r->done = true;
    }
    cv.notify_all();
  }
}

extern "C" {

mlcc_status mlcc_server_create(mlcc_context *ctx, const mlcc_server_opts *opts,
                               mlcc_server **out) {
  if (!ctx || !out) return MLCC_E_ARG;
  auto *s = new mlcc_server();
  s->ctx = ctx;
  size_t max_queue = 1024;
  uint64_t budget = 0, host_budget = 0;
  if (opts) {
    if (opts->max_slots > 0) s->max_slots = opts->max_slots;
    if (opts->max_queue > 0) max_queue = (size_t)opts->max_queue;
    budget = opts->hbm_budget;
    host_budget = opts->host_budget;
  }
  if (budget == 0) budget = ctx->al.budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipSetDevice(ctx->device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      delete s;
      return MLCC_E_DEVICE;
    }
    // blocks the context holds idle or cached count as free: they are
    // returned to the device when the lanes need the memory
    budget = (uint64_t)((fr + ctx->al.reusable()) * 0.9);
  }
  if (host_budget == 0) {
    const long pages = sysconf(_SC_PHYS_PAGES), page = sysconf(_SC_PAGE_SIZE);
    host_budget = pages > 0 && page > 0 ? (uint64_t)pages * (uint64_t)page / 4 : (16ull << 30);
  }
  s->adm = std::make_unique<Admission<Request>>(budget, host_budget, max_queue);
  for (int i = 0; i < s->max_slots; ++i) {
    auto lane = std::make_unique<Lane>();
    lane->al.root = &ctx->al;
    lane->al.device = ctx->device;
    lane->ex.al = &lane->al;
    lane->ex.bf16_map = &ctx->bf16_map;
    const bool ok =
        hipStreamCreateWithFlags(&lane->ex.stream, hipStreamNonBlocking) == hipSuccess &&
        hipHostMalloc((void **)&lane->ex.pinned, 512 * sizeof(double), hipHostMallocDefault) ==
            hipSuccess;
    lane->al.stream = lane->ex.stream;
    s->lanes.push_back(std::move(lane));
    if (!ok) {
      (void)hipGetLastError();
      for (auto &l : s->lanes) {
        if (l->ex.stream) (void)hipStreamDestroy(l->ex.stream);
        if (l->ex.pinned) (void)hipHostFree(l->ex.pinned);
      }
      delete s;
      return MLCC_E_DEVICE;
    }
  }
  for (auto &l : s->lanes) ctx->al.attach(&l->al);
  for (auto &l : s->lanes) s->workers.emplace_back(&mlcc_server::work, s, l.get());
  ctx->refs.fetch_add(1);  // dropped by mlcc_server_destroy
  *out = s;
  return MLCC_OK;
}

mlcc_status mlcc_server_destroy(mlcc_server *s) {
  if (!s) return MLCC_E_ARG;
  if (s->adm) {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &item : s->adm->stop()) {
      s->table.erase(item.req->ticket);
      delete item.req;
    }
  }
  s->cv.notify_all();
  for (auto &t : s->workers) t.join();
  for (auto &kv : s->table) delete kv.second;
  for (auto &l : s->lanes) {
    if (l->ex.stream) (void)hipStreamSynchronize(l->ex.stream);
    l->ex.work.release();
    l->ex.red.release();
    l->ex.planes.release();
    l->al.quiesce();
    s->ctx->al.detach(&l->al);
    if (l->ex.stream) (void)hipStreamDestroy(l->ex.stream);
    if (l->ex.pinned) (void)hipHostFree(l->ex.pinned);
  }
  mlcc_context *ctx = s->ctx;
  delete s;
  context_unref(ctx);
  return MLCC_OK;
}

mlcc_status mlcc_submit(mlcc_server *s, const mlcc_problem_desc *desc, int32_t n_roots,
                        const mlcc_solver_opts *gs, const mlcc_solver_opts *es, uint64_t *ticket) {
  if (!s || !desc || !gs || !es || !ticket) return MLCC_E_ARG;
  if (n_roots < 1 || gs->tol <= 0 || es->tol <= 0) return MLCC_E_ARG;
  try {
    validate_desc(desc);
  } catch (const Error &e) {
    return e.code;
  }
  if (n_roots > (int64_t)desc->n_occ * desc->n_vir) return MLCC_E_ARG;
  auto r = std::make_unique<Request>();
  r->desc = *desc;
  r->n_roots = n_roots;
  r->gs = *gs;
  r->es = *es;
  r->footprint = mlcc_request_footprint(desc, n_roots, es);
  const int64_t n = (int64_t)desc->n_occ + desc->n_vir;
  r->host_bytes = sizeof(double) * ((uint64_t)n + (desc->fock ? (uint64_t)(n * n) : 0) +
                                    ((desc->flags & MLCC_SYNTH_L) ? 0 : (uint64_t)desc->n_chol * n * n));
  auto status_of = [](AdmitStatus a) -> mlcc_status {
    switch (a) {
      case AdmitStatus::ok: return MLCC_OK;
      case AdmitStatus::too_large_hbm:
      case AdmitStatus::too_large_host: return MLCC_E_OOM;
      case AdmitStatus::busy: return MLCC_E_BUSY;
      default: return MLCC_E_STATE;
    }
  };
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const AdmitStatus a = s->adm->reserve(r->footprint, r->host_bytes);
    if (a != AdmitStatus::ok) return status_of(a);
  }
  auto cancel = [&](mlcc_status st) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->adm->cancel(r->host_bytes);
    return st;
  };
  // copy the inputs (host or device memory) before returning
  auto copy_in = [&](std::vector<double> &dst, const double *src, int64_t cnt) -> bool {
    dst.resize(cnt);
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, src) == hipSuccess && at.type == hipMemoryTypeDevice)
      return hipMemcpy(dst.data(), src, cnt * sizeof(double), hipMemcpyDeviceToHost) ==
             hipSuccess;
    (void)hipGetLastError();
    std::memcpy(dst.data(), src, cnt * sizeof(double));
    return true;
  };
  try {
    if (!copy_in(r->eps, desc->eps, n)) return cancel(MLCC_E_DEVICE);
    if (desc->fock && !copy_in(r->fock, desc->fock, n * n)) return cancel(MLCC_E_DEVICE);
    if (!(desc->flags & MLCC_SYNTH_L) && !copy_in(r->L, desc->L, (int64_t)desc->n_chol * n * n))
      return cancel(MLCC_E_DEVICE);
  } catch (const std::bad_alloc &) {
    return cancel(MLCC_E_OOM);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const AdmitStatus a = s->adm->enqueue(r.get(), r->footprint, r->host_bytes);
    if (a != AdmitStatus::ok) {
      s->adm->cancel(r->host_bytes);
      return status_of(a);
    }
    Request *q = r.release();
    q->ticket = s->next_ticket++;
    q->res.t_submit = now_s(s->t0);
    *ticket = q->ticket;
    s->table[q->ticket] = q;
  }
  s->cv.notify_all();
  return MLCC_OK;
}

mlcc_status mlcc_poll(mlcc_server *s, uint64_t ticket, mlcc_result *out) {
  if (!s || !out) return MLCC_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->table.find(ticket);
  if (it == s->table.end()) return MLCC_E_ARG;
  Request *r = it->second;
  if (!r->done) return MLCC_PENDING;
  *out = r->res;
  s->table.erase(it);
  delete r;
  return MLCC_OK;
}

}  // extern "C"
