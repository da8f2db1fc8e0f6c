// MLCC2 / MLCCSD model layer: the Omega vector, the energy and the Jacobian
// transformation, each written as a sequence of GEMM-engine calls and a few
// element-wise kernels (Sec. 2.1 and Appendix A of Folkestad et al.).
//
// Operand type T is double (MLCC_FP64) or float (MLCC_FP32, MLCC_BF16X3) for everything
// contracted over Cholesky vectors; Fock matrices, amplitudes, residuals,
// transformed vectors and energies are FP64.
//
// Layout in HBM (n = O + V, J Cholesky vectors, M = o*v active pairs):
//   L, Lt      [J][n][n]   Cholesky vectors and their X1 transform
//   Lvo0, Lai  [J][M]      packed active L_ai (untransformed) and L~_ai (MLCCSD)
//   LaiT       [M][J]      L~_ai pair-major (MLCC2)
//   LvoJ       [J+1][o][v] L^K_bj occupied-major (row J: F~_jb), the reduction
//                          operand of the pair-blocked Z contractions
//   Z          [J(+1)][M]  Z^K_ai = sum_bj u_ai,bj L^K_bj  (shared by Omega_1
//                          and the energy; row J: sum_bj u_ai,bj F~_jb)
//   g, u       [M][M]      g~_aibj and u = 2x - x(i<->j), where stored (below)
//   amp, om    [n1 (+M*M)] (t1 | MLCCSD t2) and (Omega_1 | Omega_2)
//   s2, o2     [M][M]      MLCC2 s2 and Omega_2, only when given or asked for
//
// MLCC2 with the analytic s2 (the ground state, the Jacobian at its solution)
// never stores g~ nor any other M x M array of the ground state: the doubles
// are built per occupied-pair block (I, J), I <= J, of o_b occupied indices
// each (rows (i in I, a), columns (j in J, b)):
//   s_IJ = -L~_I^T L~_J / eps   (one GEMM; FP64 denominator in its epilogue)
//   u_IJ = 2 s_IJ - s_IJ(i<->j) and u_JI = u_IJ^T (one LDS-tiled kernel: the
//          exchange partner of every element lies in the same block)
//   Z_I += L_J u_IJ^T, Z_J += L_I u_JI^T   (two GEMMs)
// which builds the upper pair-triangle of g~ only.  The effective Jacobian
// transformation treats c2 = P[L~ dL~] / (w - eps) the same way.
#include "problem.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

namespace mlcc {

// Occupied indices per pair block: nz blocks of (o_b v)^2 values in FP64 (two
// buffers) and of u in the operand type (two buffers) within kPairBlockBytes,
// balanced so that the blocks along the occupied index are of (nearly) equal
// size rather than leaving a small last block.
int pair_block_occ(int o, int v, int nz, int tsize) {
  if (o <= 0) return 1;
  const double per = (double)nz * (16.0 + 2.0 * (double)tsize);
  const double rows = std::floor(std::sqrt(kPairBlockBytes / per));
  const int cap = (int)std::max(1.0, std::min((double)o, std::floor(rows / std::max(v, 1))));
  const int blocks = (o + cap - 1) / cap;
  return (o + blocks - 1) / blocks;
}

namespace {
// Capacity of a block for a request of n bytes (plus slack): 4 KiB granules
// below 2 MiB, 2 MiB granules above, so that repeated sizes find their blocks.
size_t block_capacity(size_t n) {
  const size_t g = n < (2u << 20) ? (4u << 10) : (2u << 20);
  return (n + g - 1) / g * g;
}
// A cached block of capacity cap serves a request needing want bytes when
// it is at most 1.5 times as large: blocks of similar sizes are reused from
// request to request, but a large block (the FP64 staging copy of L, say) is
// not spent on a request of half its size, which would hold the difference
// idle for the rest of the solve.  Measured on the 256-request serving
// stream and on its largest requests alone: with up to 2x the largest
// request held 32 GB against its 26 GB footprint estimate; with at most
// 1.25x (or 32 MiB) fewer blocks were reused and the stream ran slower.
bool fits(size_t cap, size_t want) { return cap >= want && 2 * cap <= 3 * want; }
}  // namespace

void *Alloc::get(size_t bytes) {
  const size_t want = block_capacity(bytes + kSlack);
  void *p = nullptr;
  size_t cap = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.lower_bound(want);
    if (it != cache.end() && fits(it->first, want)) {
      cap = it->first;
      p = it->second;
      cache.erase(it);
    }
  }
  Alloc *r = root;
  if (!p) {
    std::lock_guard<std::mutex> lk(r->mu);
    auto it = r->idle.lower_bound(want);
    if (it != r->idle.end() && fits(it->first, want)) {
      cap = it->first;
      p = it->second;
      r->idle.erase(it);
    }
  }
  if (!p) {
    bool over;
    {
      std::lock_guard<std::mutex> lk(r->mu);
      over = r->budget && r->held + want > r->budget;
    }
    if (over) {
      reclaim(want);
      std::lock_guard<std::mutex> lk(r->mu);
      over = r->budget && r->held + want > r->budget;
    }
    if (over) r->reclaim_all(want);
    {
      std::lock_guard<std::mutex> lk(r->mu);
      if (r->budget && r->held + want > r->budget)
        throw Error{MLCC_E_OOM, "HBM budget exceeded: need " + std::to_string(want) + " bytes, " +
                                    std::to_string(r->budget - r->held) + " left"};
      r->held += want;  // reserved while the allocation is made
    }
    // out of device memory: free idle blocks (no pending work uses them),
    // then this stream's cached blocks, then those the other lanes of the
    // context cached while their requests run, each time only about what
    // the allocation needs (with room for the runtime's own allocations)
    const size_t need = want + ((size_t)256 << 20);
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      r->trim(need);
      e = hipMalloc(&p, want);
    }
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      reclaim(need);
      e = hipMalloc(&p, want);
    }
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      r->reclaim_all(need);
      e = hipMalloc(&p, want);
    }
    // a lane of a server: the other lanes' requests return their memory when
    // they finish; wait for that (up to about a minute) before failing
    for (int attempt = 0; e == hipErrorOutOfMemory && r != this && attempt < 600; ++attempt) {
      (void)hipGetLastError();
      std::this_thread::sleep_for(std::chrono::milliseconds(100));
      r->reclaim_all(need);
      e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      std::lock_guard<std::mutex> lk(r->mu);
      r->held -= want;
      throw Error{e == hipErrorOutOfMemory ? MLCC_E_OOM : MLCC_E_DEVICE,
                  std::string("hipMalloc: ") + hipGetErrorString(e)};
    }
    cap = want;
  }
  std::lock_guard<std::mutex> lk(r->mu);
  r->live[reinterpret_cast<uintptr_t>(p)] = cap;
  r->used += cap;
  return p;
}

void Alloc::put(void *p, size_t) {
  Alloc *r = root;
  size_t cap = 0;
  {
    std::lock_guard<std::mutex> lk(r->mu);
    auto it = r->live.find(reinterpret_cast<uintptr_t>(p));
    if (it == r->live.end()) return;
    cap = it->second;
    r->live.erase(it);
    r->used -= cap;
  }
  std::lock_guard<std::mutex> lk(mu);
  cache.emplace(cap, p);
}

void Alloc::quiesce() {
  std::multimap<size_t, void *> blocks;
  {
    std::lock_guard<std::mutex> lk(mu);
    blocks.swap(cache);
  }
  std::lock_guard<std::mutex> lk(root->mu);
  root->idle.insert(blocks.begin(), blocks.end());
}

void Alloc::trim(size_t need) {
  std::vector<std::pair<size_t, void *>> blocks;
  {
    std::lock_guard<std::mutex> lk(mu);
    size_t sum = 0;
    while (!idle.empty() && (need == 0 || sum < need)) {
      auto it = std::prev(idle.end());  // the largest
      sum += it->first;
      blocks.emplace_back(it->first, it->second);
      idle.erase(it);
    }
  }
  size_t freed = 0;
  for (auto &b : blocks) {
    (void)hipFree(b.second);
    freed += b.first;
  }
  std::lock_guard<std::mutex> lk(mu);
  held -= freed;
}

void Alloc::reclaim(size_t need) {
  if (stream) (void)hipStreamSynchronize(stream);
  quiesce();
  root->trim(need);
}

size_t Alloc::reusable() {
  std::lock_guard<std::mutex> lk(mu);
  size_t n = 0;
  for (auto &b : idle) n += b.first;
  for (auto &b : cache) n += b.first;
  return n;
}

void Alloc::put_idle(void *p) {
  Alloc *r = root;
  if (stream) (void)hipStreamSynchronize(stream);
  std::lock_guard<std::mutex> lk(r->mu);
  auto it = r->live.find(reinterpret_cast<uintptr_t>(p));
  if (it == r->live.end()) return;
  const size_t cap = it->second;
  r->live.erase(it);
  r->used -= cap;
  r->idle.emplace(cap, p);
}

void Alloc::reclaim_all(size_t need) {
  std::vector<Alloc *> all;
  {
    std::lock_guard<std::mutex> lk(mu);
    all = lanes;
  }
  all.push_back(this);
  for (Alloc *a : all) {
    // every block in the cache was released after the work that used it was
    // enqueued on the lane's stream: once that stream has drained up to now,
    // no pending work uses them
    std::multimap<size_t, void *> blocks;
    {
      std::lock_guard<std::mutex> lk(a->mu);
      blocks.swap(a->cache);
    }
    if (blocks.empty()) continue;
    if (a->stream) (void)hipStreamSynchronize(a->stream);
    std::lock_guard<std::mutex> lk(mu);
    idle.insert(blocks.begin(), blocks.end());
  }
  trim(need);
}

void Alloc::attach(Alloc *lane) {
  std::lock_guard<std::mutex> lk(mu);
  lanes.push_back(lane);
}

void Alloc::detach(Alloc *lane) {
  std::lock_guard<std::mutex> lk(mu);
  lanes.erase(std::remove(lanes.begin(), lanes.end(), lane), lanes.end());
}

void Alloc::release_all() {
  quiesce();
  trim();
}

bool Alloc::owns(const void *p) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  Alloc *r = root;
  std::lock_guard<std::mutex> lk(r->mu);
  auto it = r->live.upper_bound(a);
  if (it == r->live.begin()) return false;
  --it;
  return a < it->first + it->second - kSlack;
}

}  // namespace mlcc

using namespace mlcc;

double mlcc_problem::fetch(const double *dev) {
  double *h = ex->pinned;
  MLCC_HIP(hipMemcpyAsync(h, dev, sizeof(double), hipMemcpyDeviceToHost, ex->stream));
  MLCC_HIP(hipStreamSynchronize(ex->stream));
  return h[0];
}

void mlcc_problem::fetch_n(const double *dev, double *host, int n) {
  MLCC_HIP(hipMemcpyAsync(host, dev, sizeof(double) * n, hipMemcpyDeviceToHost, ex->stream));
  MLCC_HIP(hipStreamSynchronize(ex->stream));
}

// ---------------------------------------------------------------------------
// setup: inputs, core Hamiltonian h = diag(eps) - G(D_HF), denominators
// ---------------------------------------------------------------------------
template <typename T>
void mlcc_problem::setup_t(const double *Lsrc, bool dev, const uint64_t *synth_seed) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O;
  const size_t nL = (size_t)J * n2;
  // FP64 staging copy of L (the input), used for h and converted if FP32
  DBuf L64;
  double *L64p;
  if (sizeof(T) == 8) {
    L.alloc(al, nL * sizeof(double));
    L64p = L.as<double>();
  } else {
    L64.alloc(al, nL * sizeof(double));
    L64p = L64.as<double>();
  }
  if (synth_seed)
    k::synth_cholesky(x, L64p, J, n, d.O, d.V, *synth_seed);
  else
    MLCC_HIP(hipMemcpyAsync(L64p, Lsrc, nL * sizeof(double),
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, x.stream));
  // h = diag(eps) - 2 sum_K L^K d^K + sum_{K,I} L^K_pI L^K_Iq   (FP64); the
  // diagonal is added by the caller
  h.alloc(al, n2 * sizeof(double));
  k::fill(x, h.as<double>(), n2, 0.0);
  dK.alloc(al, J * sizeof(double));
  k::occ_trace<double>(x, J, n, d.O, L64p, dK.as<double>());
  {
    // exchange: h += sum_r L^r[:, occ] L^r[occ, :]
    G(n, n, O, J).A(L64p, n, 1, n2).B(L64p, n, 1, n2).C(h.as<double>(), n, 1, 0, 1.0, 1.0)
        .run(x, Prec::F64, true);
    // Coulomb: row p: h[p][:] += -2 sum_K d^K L^K[p][:]
    G(1, n, J, 1, n).A(dK.p, 0, 1, 0, 0).B(L64p, n2, 1, 0, n).C(h.as<double>(), 0, 1, n, -2.0,
                                                                  1.0)
        .run(x, Prec::F64, true);
  }
  if (sizeof(T) == 4) {
    L.alloc(al, nL * sizeof(float));
    k::convert<float, double>(x, L.as<float>(), L64p, nL);
    // the staging copy (twice the bytes of L) becomes idle in the context
    // now rather than waiting in this stream's cache, where nothing of this
    // problem would reuse it
    L64.release_idle();
  }
  // packed active L_ai (= L_ia): Lvo0[K][a*o+i] = L^K[O+a][i]
  if (d.M > 0) {
    // one spare row after the J rows: the Jacobian puts F~_jb there, so that
    // the u(c2) contraction with L_bj also yields sum_bj u_aibj F~_jb
    Lvo0.alloc(al, (size_t)(J + 1) * d.M * sizeof(T));
    k::pack2d<T, T>(x, off<T>(Lvo0), off<T>(L, (int64_t)O * n), J, n2, d.v, d.o, n);
    if (model == MLCC_MLCC2) {
      // the same occupied-major, LvoJ[K][j*v+b] = L^K[O+b][j] (spare row J likewise)
      LvoJ.alloc(al, (size_t)(J + 1) * d.M * sizeof(T));
      k::pack2d_t<T, T>(x, off<T>(LvoJ), off<T>(L, (int64_t)O * n), J, n2, d.v, d.o, n);
    }
  }
  MLCC_HIP(hipStreamSynchronize(x.stream));
}

namespace {
__global__ void k_add_diag(int64_t n, const double *eps, double *h) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    h[i * n + i] += eps[i];
}
}  // namespace

void mlcc_problem::setup(const mlcc_problem_desc &desc) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  d.O = desc.n_occ;
  d.V = desc.n_vir;
  d.J = desc.n_chol;
  d.n = d.O + d.V;
  model = desc.model;
  prec = desc.precision;
  if (model == MLCC_CCS) {
    d.o = 0;
    d.v = 0;
  } else {
    d.o = desc.n_occ_act;
    d.v = desc.n_vir_act;
  }
  // three-level MLCCSD runs as MLCCSD over the active space whose CCSD-level
  // doubles projections are restricted to the CCSD space (ot, vt)
  d.ot = d.o;
  d.vt = d.v;
  if (model == MLCC_MLCCSD3) {
    model = MLCC_MLCCSD;
    d.ot = desc.n_occ_ccsd;
    d.vt = desc.n_vir_ccsd;
  }
  d.M = (int64_t)d.o * d.v;
  d.n1 = (int64_t)d.O * d.V;
  d.n2 = (int64_t)d.n * d.n;
  tsize = prec == MLCC_FP64 ? 8 : 4;

  hipPointerAttribute_t at;
  auto is_dev = [&](const void *p) {
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return at.type == hipMemoryTypeDevice;
  };
  eps.alloc(al, d.n * sizeof(double));
  MLCC_HIP(hipMemcpyAsync(eps.p, desc.eps, d.n * sizeof(double),
                          is_dev(desc.eps) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          x.stream));
  eps_vo.alloc(al, d.n1 * sizeof(double));
  eps_ai.alloc(al, std::max<int64_t>(d.M, 1) * sizeof(double));
  k::denominators(x, d.O, d.V, d.o, d.v, eps.as<double>(), eps_ai.as<double>(),
                  eps_vo.as<double>());
  eps_aiT.alloc(al, std::max<int64_t>(d.M, 1) * sizeof(double));
  if (d.M > 0)
    k::pack2d_t<double, double>(x, eps_aiT.as<double>(), eps_ai.as<double>(), 1, 0, d.v, d.o, d.o);
  res.alloc(al, 64 * sizeof(double));
  // NaN/Inf in eps
  k::nonfinite(x, d.n, eps.as<double>(), res.as<double>());
  MLCC_REQUIRE(fetch(res.as<double>()) == 0.0, MLCC_E_NUMERIC, "non-finite orbital energy");

  const bool synth = (desc.flags & MLCC_SYNTH_L) != 0;
  const bool ldev = !synth && is_dev(desc.L);
  const uint64_t *sp = synth ? &desc.seed : nullptr;
  if (prec == MLCC_FP64) setup_t<double>(desc.L, ldev, sp);
  else setup_t<float>(desc.L, ldev, sp);
  // h += F  (the setup above accumulated -G into a zeroed h): diag(eps), or
  // the given Fock matrix (kept for mlcc_cnto)
  if (desc.fock) {
    fock.alloc(al, d.n2 * sizeof(double));
    MLCC_HIP(hipMemcpyAsync(fock.p, desc.fock, d.n2 * sizeof(double),
                            is_dev(desc.fock) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            x.stream));
    k::nonfinite(x, d.n2, fock.as<double>(), res.as<double>());
    MLCC_REQUIRE(fetch(res.as<double>()) == 0.0, MLCC_E_NUMERIC, "non-finite Fock matrix");
    k::lincomb<double>(x, d.n2, 1.0, h.as<double>(), 1.0, fock.as<double>(), h.as<double>());
  } else {
    hipLaunchKernelGGL(k_add_diag, dim3(64), dim3(256), 0, x.stream, (int64_t)d.n,
                       eps.as<double>(), h.as<double>());
    MLCC_HIP(hipGetLastError());
  }
  // NaN/Inf in L shows up in h
  k::nonfinite(x, d.n2, h.as<double>(), res.as<double>());
  MLCC_REQUIRE(fetch(res.as<double>()) == 0.0, MLCC_E_NUMERIC, "non-finite Cholesky vectors");

  const int64_t nd = model == MLCC_MLCCSD ? d.M * d.M : 0;
  amp.alloc(al, (size_t)(d.n1 + nd) * sizeof(double));
  MLCC_HIP(hipMemsetAsync(amp.p, 0, amp.bytes, x.stream));
  om.alloc(al, amp.bytes);
  MLCC_HIP(hipStreamSynchronize(x.stream));
}

// ---------------------------------------------------------------------------
// X1 basis (Appendix A): L~ = (1 - T) L (1 + T), T[A][I] = t_AI, blockwise
//   L~_ov = L_ov
//   L~_oo = L_oo + L_ov t
//   L~_vv = L_vv - t L_ov
//   L~_vo = L_vo + L_vv t - t L~_oo
// and the Fock matrix F~ = h~ + sum_I (2 g~_pqII - g~_pIIq).
// ---------------------------------------------------------------------------
namespace {
template <typename T>
void x1_blocks(Exec &x, Prec p, const Dims &d, const T *src, T *dst, int64_t Z, const T *t) {
  const int64_t n = d.n, n2 = d.n2, O = d.O, V = d.V;
  const bool o64 = sizeof(T) == 8;
  // ov copy: C = 1 * Cin with an empty reduction
  G(O, V, 0, 1, Z).C(dst + O, n, 1, n2, 0.0, 1.0, src + O).run(x, p, o64);
  G(O, O, V, 1, Z).A(src + O, n, 1, 0, n2).B(t, O, 1, 0, 0).C(dst, n, 1, n2, 1.0, 1.0, src)
      .run(x, p, o64);
  G(V, V, O, 1, Z).A(t, O, 1, 0, 0).B(src + O, n, 1, 0, n2)
      .C(dst + O * n + O, n, 1, n2, -1.0, 1.0, src + O * n + O).tag("x1_vv").run(x, p, o64);
  G(V, O, V, 1, Z).A(src + O * n + O, n, 1, 0, n2).B(t, O, 1, 0, 0)
      .C(dst + O * n, n, 1, n2, 1.0, 1.0, src + O * n).tag("x1_vo").run(x, p, o64);
  G(V, O, O, 1, Z).A(t, O, 1, 0, 0).B(dst, n, 1, 0, n2)
      .C(dst + O * n, n, 1, n2, -1.0, 1.0, dst + O * n).run(x, p, o64);
}
}  // namespace

template <typename T> void mlcc_problem::dress_t(bool full_fock) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O, V = d.V, o = d.o, v = d.v;
  const Prec p = gemm_prec<T>();
  t1T.ensure(al, d.n1 * sizeof(T));
  if (sizeof(T) == 8) MLCC_HIP(hipMemcpyAsync(t1T.p, t1(), d.n1 * 8, hipMemcpyDeviceToDevice, x.stream));
  else k::convert<float, double>(x, t1T.as<float>(), t1(), d.n1);
  Lt.ensure(al, (size_t)J * n2 * sizeof(T));
  x1_blocks<T>(x, gemm_prec<T>(), d, off<T>(L), off<T>(Lt), J, off<T>(t1T));
  ht.ensure(al, n2 * sizeof(double));
  x1_blocks<double>(x, Prec::F64, d, h.as<double>(), ht.as<double>(), 1, t1());
  // F~ = h~ + 2 sum_K L~^K d~^K - sum_{K,I} L~^K_pI L~^K_Iq
  Ft.ensure(al, n2 * sizeof(double));
  MLCC_HIP(hipMemcpyAsync(Ft.p, ht.p, n2 * sizeof(double), hipMemcpyDeviceToDevice, x.stream));
  dK.ensure(al, J * sizeof(double));
  dKT.ensure(al, J * sizeof(T));
  k::occ_trace<T>(x, J, n, (int)O, off<T>(Lt), dK.as<double>());
  k::convert<T, double>(x, off<T>(dKT), dK.as<double>(), J);
  const T *lt = off<T>(Lt);
  double *F = Ft.as<double>();
  auto fock_block = [&](int64_t r0, int64_t nr, int64_t c0, int64_t nc) {
    if (nr <= 0 || nc <= 0) return;
    G(nr, nc, O, J).A(lt + r0 * n, n, 1, n2).B(lt + c0, n, 1, n2)
        .C(F + r0 * n + c0, n, 1, 0, -1.0, 1.0).tag("fock_exch").run(x, p, true);
    G(1, nc, J, 1, nr).A(off<T>(dKT), 0, 1, 0, 0).B(lt + r0 * n + c0, n2, 1, 0, n)
        .C(F + r0 * n + c0, 0, 1, n, 2.0, 1.0).run(x, p, true);
  };
  if (full_fock) {
    fock_block(0, n, 0, n);
  } else {
    fock_block(O, V, 0, O);   // F~_AI
    fock_block(0, o, O, v);   // F~_jb (active)
    if (model == MLCC_MLCCSD) {
      fock_block(O, v, O, v);  // F~_bc (active)
      fock_block(0, o, 0, o);  // F~_kj (active)
    }
  }
  fock_full = full_fock;
}

// Doubles-dependent quantities at given doubles (MLCC2 with an independent s2,
// MLCCSD t2): L~_ai packed, g~_aibj (MLCC2, stored for Omega_2 = g~ + eps s),
// u = 2x - x(i<->j) and Z^K_ai = sum_bj u_ai,bj L^K_bj.
template <typename T> void mlcc_problem::doubles_mlcc2_t() {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O, M = d.M;
  const Prec p = gemm_prec<T>();
  u.ensure(al, (size_t)M * M * sizeof(T));
  u_occ = false;
  if (model == MLCC_MLCC2) {
    // L~_ai pair-major, LaiT[ai][K]: the reduction index of g~ and of the
    // Jacobian's doubles block is contiguous (split BF16 products need it)
    LaiT.ensure(al, (size_t)J * M * sizeof(T));
    const int64_t nn[4] = {1, d.v, d.o, J}, ss[4] = {0, n, 1, n2};
    k::permute4<T, T>(x, off<T>(LaiT), off<T>(Lt, O * n), nn, ss, 1.0, 0.0);
    g.ensure(al, (size_t)M * M * sizeof(double));
    // g~_ai,bj = sum_K L~^K_ai L~^K_bj
    G(M, M, J).A(off<T>(LaiT), J, 1).B(off<T>(LaiT), 1, J).C(g.p, M, 1).tag("g_aibj")
        .run(x, p, true);
    k::u_of<T>(x, d.o, d.v, x2(), off<T>(u));
  } else {
    // MLCCSD: L~_ai K-major, Lai[K][ai] (its integral blocks read it so)
    Lai.ensure(al, (size_t)J * M * sizeof(T));
    k::pack2d<T, T>(x, off<T>(Lai), off<T>(Lt, O * n), J, n2, d.v, d.o, n);
    k::u_of<T>(x, d.o, d.v, x2(), off<T>(u));
  }
  // Z^K_ai = sum_bj L^K_bj u_bj,ai, with u read through its pair symmetry
  // (u_bj,ai = u_ai,bj) so that both operands run along the reduction index
  Z.ensure(al, (size_t)J * M * sizeof(T));
  G(J, M, M).A(off<T>(Lvo0), M, 1).B(off<T>(u), 1, M).C(Z.p, M, 1).tag("Z_uL").run(x, p, sizeof(T) == 8);
}

int mlcc_problem::occ_batch(int nz) const {
  if (ctx->pair_occ > 0) return std::min(ctx->pair_occ, d.o);
  return pair_block_occ(d.o, d.v, nz, (int)tsize);
}

// MLCC2 doubles with the analytic s2 (App. A, MLCC2 Omega vector: the
// doubles equation is solved by s_aibj = -g~_aibj / eps_aibj in the
// semicanonical basis), built per occupied-pair block and contracted at once
// into Z^K_ai = sum_bj u_ai,bj L^K_bj (row J: sum_bj u_ai,bj F~_jb).  keep_u
// also stores u (occupied-major rows and columns) for the Jacobian; want_s
// writes s to the full a-major s2 array.
template <typename T> void mlcc_problem::doubles_pairblocks_t(bool keep_u) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O, M = d.M, o = d.o, v = d.v;
  const Prec p = gemm_prec<T>();
  // L~_ai pair-major, LaiT[ai][K] (reduction index contiguous)
  LaiT.ensure(al, (size_t)J * M * sizeof(T));
  const int64_t nn[4] = {1, v, o, J}, ss[4] = {0, n, 1, n2};
  k::permute4<T, T>(x, off<T>(LaiT), off<T>(Lt, O * n), nn, ss, 1.0, 0.0);
  // F~_jb (occupied-major) in the spare row of LvoJ
  k::pack2d<T, double>(x, off<T>(LvoJ, J * M), Ft.as<double>() + O, 1, 0, o, v, n);
  Z.ensure(al, (size_t)(J + 1) * M * sizeof(T));
  MLCC_HIP(hipMemsetAsync(Z.p, 0, (size_t)(J + 1) * M * sizeof(T), x.stream));
  g.release();  // no g~ is kept
  const int ob = occ_batch(1);
  const int64_t Rm = (int64_t)std::min<int64_t>(ob, o) * v;
  pbX.ensure(al, (size_t)Rm * Rm * sizeof(double));
  if (keep_u) {
    u.ensure(al, (size_t)M * M * sizeof(T));
    u_occ = true;
  } else {
    pbU1.ensure(al, (size_t)Rm * Rm * sizeof(T));
    pbU2.ensure(al, (size_t)Rm * Rm * sizeof(T));
  }
  if (want_s) ensure_doubles();
  const T *lai = off<T>(LaiT);
  const double *eT = eps_aiT.as<double>();
  for (int i0 = 0; i0 < o; i0 += ob) {
    const int ni = (int)std::min<int64_t>(ob, o - i0);
    const int64_t RI = (int64_t)ni * v;
    for (int j0 = i0; j0 < o; j0 += ob) {
      const int nj = (int)std::min<int64_t>(ob, o - j0);
      const int64_t RJ = (int64_t)nj * v;
      const bool diag = j0 == i0;
      // s[(i,a)][(j,b)] = -sum_K L~^K_ai L~^K_bj / (e_a - e_i + e_b - e_j)
      G(RI, RJ, J).A(lai + i0 * J, o * J, 1).Mhi(v, J, v * RJ).B(lai + j0 * J, 1, o * J)
          .Nhi(v, J, v).C(pbX.p, RJ, 1, 0, -1.0, 0.0).den(eT + i0 * v, eT + j0 * v)
          .tag("g_aibj").run(x, p, true);
      T *u1 = keep_u ? off<T>(u, i0 * v * M + j0 * v) : off<T>(pbU1);
      T *u2 = diag ? nullptr : (keep_u ? off<T>(u, j0 * v * M + i0 * v) : off<T>(pbU2));
      const int64_t l1 = keep_u ? M : RJ, l2 = keep_u ? M : RI;
      k::u_pairblock<T>(x, (int)o, (int)v, ni, nj, pbX.as<double>(), RJ, 0, u1, l1, u2, l2, 0, 1,
                        want_s ? x2() : nullptr, i0, j0);
      // Z^K_ai (i in I) += sum_(j,b) L^K_bj u_IJ; rows K and the F~ row J
      G(J + 1, RI, RJ).A(off<T>(LvoJ, j0 * v), M, 1).B(u1, 1, l1).Nhi(v, v * l1, 1)
          .C(off<T>(Z, i0), M, o, 0, 1.0, 1.0).tag("Z_uL").run(x, p, sizeof(T) == 8);
      if (!diag)
        G(J + 1, RJ, RI).A(off<T>(LvoJ, i0 * v), M, 1).B(u2, 1, l2).Nhi(v, v * l2, 1)
            .C(off<T>(Z, j0), M, o, 0, 1.0, 1.0).tag("Z_uL").run(x, p, sizeof(T) == 8);
    }
  }
}

// Omega_AI += [I act] sum_Kb L~^K_Ab Z^K_bi - [A act] sum_Kk Z^K_ak L~^K_kI
//           + [A,I act] sum_bj u_ai,bj F~_jb    (Appendix A, MLCC2 Omega vector)
// optionally starting from F~_AI.  Also the singles-from-doubles part of the
// Jacobian transformation when Zb/ub come from a trial vector.
template <typename T>
void mlcc_problem::omega_singles_t(const void *Zb, const void *ub, double *om1, bool add_fock) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O, V = d.V, o = d.o, v = d.v, M = d.M;
  const Prec p = gemm_prec<T>();
  if (add_fock) k::pack2d<double, double>(x, om1, Ft.as<double>() + O * n, 1, 0, V, O, n);
  if (M == 0 || Zb == nullptr) return;
  const T *lt = off<T>(Lt);
  const T *zb = static_cast<const T *>(Zb);
  G(V, o, v, J).A(lt + O * n + O, n, 1, n2).B(zb, o, 1, M).C(om1, O, 1, 0, 1.0, 1.0)
      .run(x, p, true);
  G(v, O, o, J).A(zb, o, 1, M).B(lt, n, 1, n2).C(om1, O, 1, 0, -1.0, 1.0).run(x, p, true);
  if (!ub) {
    // the pair-blocked doubles carry sum_bj u_aibj F~_jb in row J of Z
    k::acc3d<T>(x, 1, v, o, 1.0, zb + J * M, 0, o, 1, om1, 0, O);
    return;
  }
  fvec.ensure(al, M * sizeof(T));
  k::pack2d_t<T, double>(x, off<T>(fvec), Ft.as<double>() + O, 1, 0, o, v, n);
  G(o, 1, M, 1, v).A(ub, M, 1, 0, o * M).B(fvec.p, 1, 0).C(om1, 1, 0, O, 1.0, 1.0)
      .run(x, p, true);
}

template <typename T> void mlcc_problem::compute_state_t(bool full_fock, bool keep_u) {
  Exec &x = *ex;
  const int64_t J = d.J, n = d.n, M = d.M, n1 = d.n1;
  dress_t<T>(full_fock);
  double *om1 = om.as<double>();
  if (has_doubles() && model == MLCC_MLCC2 && !x2_set) {
    doubles_pairblocks_t<T>(keep_u);
    omega_singles_t<T>(Z.p, nullptr, om1, true);
    if (want_om2) {
      // the analytic s2 solves the doubles equation: Omega_2 = 0
      ensure_doubles();
      MLCC_HIP(hipMemsetAsync(om2(), 0, (size_t)M * M * sizeof(double), x.stream));
    }
  } else if (has_doubles()) {
    doubles_mlcc2_t<T>();
    omega_singles_t<T>(Z.p, u.p, om1, true);
    if (model == MLCC_MLCC2)
      k::mlcc2_omega2<double>(x, M, g.as<double>(), eps_ai.as<double>(), x2(), om2());
    else
      ccsd_omega2_t<T>();
  } else {
    omega_singles_t<T>(nullptr, nullptr, om1, true);
  }
  // energy: E1 = 2 sum_K (tr Q^K)^2 - sum_K tr(Q^K Q^K), Q^K = (L_ov t)^K = L~_oo - L_oo;
  //         E2 = sum_ai,bj u_ai,bj g_ai,bj = sum_K sum_ai L^K_ai Z^K_ai
  double *r = res.as<double>();
  k::energy_singles<T>(x, J, n, d.O, off<T>(Lt), off<T>(L), r + 0);
  if (has_doubles()) k::dot_mixed<T, T>(x, J * M, off<T>(Lvo0), off<T>(Z), r + 1);
  else k::fill(x, r + 1, 1, 0.0);
  // residual norms
  k::dot(x, n1, om1, om1, r + 2);
  if (has_doubles() && (model == MLCC_MLCCSD || x2_set))
    k::dot(x, M * M, om2(), om2(), r + 3);
  else
    k::fill(x, r + 3, 1, 0.0);
  double hr[4];
  fetch_n(r, hr, 4);
  e_corr = hr[0] + hr[1];
  omega_norm = std::sqrt(hr[2] + hr[3]);
  state_valid = true;
}

#include "ccsd.inl"

void mlcc_problem::compute_state(bool full_fock, bool keep_u) {
  if (prec == MLCC_FP64) compute_state_t<double>(full_fock, keep_u);
  else compute_state_t<float>(full_fock, keep_u);
}

// ---------------------------------------------------------------------------
// Jacobian transformation (Appendix A.2), the derivative of the Omega vector:
// with dL~ = L~ C - C L~ (C[A][I] = c_AI) and dF~ likewise, the singles part is
//   CCS:   F~_AB c_BI - c_AJ F~_JI + 2 (L~^K_JB c_BJ) L~^K_AI - (L~^K_AB c_BJ) L~^K_JI
//   MLCC2: - c_AJ X_Ji - Y_aB c_BI + u_ai,ck (2 q_ck - r_ck)
//          with X_Ji = sum L~^K_Jb Z^K_bi, Y_aB = sum Z^K_ak L~^K_kB,
//          q_ck = sum_K L^K_ck (L~^K_JB c_BJ), r_ck = sum (L~^K_kB c_BJ) L~^K_Jc
//   doubles -> singles: the Omega_1 doubles terms with u -> 2c - c(i<->j)
// and the doubles part is dg~ + eps * c2 = P[(dL~^K_ai) L~^K_bj] + eps c2.
// ---------------------------------------------------------------------------
template <typename T> void mlcc_problem::prepare_jacobian_t() {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O, V = d.V, o = d.o, v = d.v, M = d.M;
  const Prec p = gemm_prec<T>();
  compute_state_t<T>(true, true);
  {
    // LooT[K][i][J] = L~^K_Ji: the occupied reduction index J contiguous for
    // the c L~_oo products of the transformation
    LooT.ensure(al, (size_t)J * O * O * sizeof(T));
    const int64_t nn[4] = {1, J, O, O}, ss[4] = {0, n2, 1, n};
    k::permute4<T, T>(x, off<T>(LooT), off<T>(Lt), nn, ss, 1.0, 0.0);
  }
  if (has_doubles()) {
    Xint.ensure(al, O * o * sizeof(T));
    Yint.ensure(al, v * V * sizeof(T));
    const T *lt = off<T>(Lt);
    G(O, o, v, J).A(lt + O, n, 1, n2).B(Z.p, o, 1, M).C(Xint.p, o, 1).run(x, p, sizeof(T) == 8);
    G(v, V, o, J).A(Z.p, o, 1, M).B(lt + O, n, 1, n2).C(Yint.p, V, 1).run(x, p, sizeof(T) == 8);
    if (model == MLCC_MLCCSD) ccsd_prepare_t<T>();
  }
  jac_ready = true;
}

void mlcc_problem::prepare_jacobian() {
  if (prec == MLCC_FP64) prepare_jacobian_t<double>();
  else prepare_jacobian_t<float>();
}

// A batch of nb vectors at once: c[vec] at c + vec*ld (singles first, then
// the doubles when c2 is present), sigma likewise.  With has_c2 false the
// vectors are singles only; then, if w_eff is finite (MLCC2), the doubles are
// eliminated, c2 = (A21 c1)/(w_eff - eps_aibj), and only sigma_1 is produced.
template <typename T>
void mlcc_problem::transform_batch_t(int nb, const double *c, int64_t ld, bool has_c2,
                                     double *sigma, double w_eff) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O, V = d.V, o = d.o, v = d.v, M = d.M;
  const int64_t n1 = d.n1, b = nb;
  const Prec p = gemm_prec<T>();
  const bool o64 = sizeof(T) == 8;
  const T *lt = off<T>(Lt);
  const double *F = Ft.as<double>();
  cT.ensure(al, b * n1 * sizeof(T));
  cTt.ensure(al, b * n1 * sizeof(T));
  T *ct = off<T>(cT);
  k::pack2d<T, double>(x, ct, c, b, ld, 1, n1, 0);
  // and transposed, ctt[vec][I][A] (the virtual index contiguous)
  T *ctt = off<T>(cTt);
  k::pack2d_t<T, double>(x, ctt, c, b, ld, V, O, O);
  const T *loot = off<T>(LooT);

  // CCS terms: F~_AB c_BI - c_AJ F~_JI + 2 (L~^K_JB c_BJ) L~^K_AI - (L~^K_AB c_BJ) L~^K_JI
  G(V, O, V, 1, b).A(F + O * n + O, n, 1, 0, 0).B(c, O, 1, 0, ld).C(sigma, O, 1, ld)
      .tag("ccs_fock").run(x, Prec::F64, true);
  G(V, O, O, 1, b).A(c, O, 1, 0, ld).B(F, n, 1, 0, 0).C(sigma, O, 1, ld, -1.0, 1.0)
      .tag("ccs_fock").run(x, Prec::F64, true);
  Xk.ensure(al, J * b * sizeof(T));
  G(J, b, V, O).A(lt + O, n2, 1, n).B(ct, O, n1, 1).C(Xk.p, b, 1).tag("ccs_Xk").run(x, p, o64);
  G(O, b, J, 1, V).A(lt + O * n, 1, n2, 0, n).B(Xk.p, b, 1).C(sigma, 1, ld, O, 2.0, 1.0)
      .tag("ccs_coul").run(x, p, true);
  // W^K[vec][i][B] = sum_J c_BJ L~^K_Ji, stored with B innermost so that the
  // reduction index of ccs_vv is contiguous; computed as rows i x columns
  // (vec, B) so that the output rows are contiguous too
  W.ensure(al, (size_t)J * b * V * O * sizeof(T));
  G(O, b * V, O, 1, J).A(loot, O, 1, 0, O * O).B(ct, 1, O, 0, 0).Nhi(V, n1, V * O)
      .C(W.p, V, 1, b * V * O).tag("ccs_W").run(x, p, o64);
  G(V, b * O, V, J).A(lt + O * n + O, n, 1, n2).B(W.p, 1, V, b * V * O).Nhi(O, V * O, ld)
      .C(sigma, O, 1, 0, -1.0, 1.0).tag("ccs_vv").run(x, p, true);
  if (!has_doubles()) return;

  // MLCC2 singles-singles terms with the ground-state u:
  //   - c_AJ X_Ji - Y_aB c_BI + u_ai,ck (2 q_ck - r_ck)
  G(V, o, O, 1, b).A(ct, O, 1, 0, n1).B(Xint.p, o, 1, 0, 0).C(sigma, O, 1, ld, -1.0, 1.0)
      .tag("jac_X").run(x, p, true);
  G(v, O, V, 1, b).A(Yint.p, V, 1, 0, 0).B(ct, O, 1, 0, n1).C(sigma, O, 1, ld, -1.0, 1.0)
      .tag("jac_Y").run(x, p, true);
  qv.ensure(al, M * b * sizeof(T));
  rv.ensure(al, M * b * sizeof(T));
  P.ensure(al, (size_t)J * o * b * O * sizeof(T));
  G(M, b, J).A(off<T>(Lvo0), 1, M).B(Xk.p, b, 1).C(qv.p, b, 1).tag("jac_q").run(x, p, o64);
  // P^K[i][vec, J] = sum_B L~^K_iB c_BJ as one launch over rows (K, i), reading
  // the transposed singles so that the reduction index is contiguous in both
  G(J * o, b * O, V).A(lt + O, n, 1).Mhi(o, n2, o * b * O).B(ctt, 1, V).Nhi(O, n1, O)
      .C(P.p, b * O, 1).tag("jac_P").run(x, p, o64);
  G(v, o * b, O, J).A(lt + O, 1, n, n2).B(P.p, 1, O, o * b * O).C(rv.p, o * b, 1)
      .tag("jac_r").run(x, p, o64);
  k::lincomb<T>(x, M * b, 2.0, off<T>(qv), -1.0, off<T>(rv), off<T>(qv));
  if (u_occ) {
    // u[(i,a)][(k,c)] occupied-major: rows (i, a), reduction c in slices k
    G(M, b, v, o).A(u.p, M, 1, v).Mhi(v, v * M, 1).B(qv.p, o * b, 1, b)
        .C(sigma, O, ld, 0, 1.0, 1.0).tag("jac_uw").run(x, p, true);
  } else {
    G(o, b, M, 1, v).A(u.p, M, 1, 0, o * M).B(qv.p, b, 1).C(sigma, 1, ld, O, 1.0, 1.0)
        .tag("jac_uw").run(x, p, true);
  }

  // singles -> doubles: dL~_ai = sum_B L~_aB c_Bi - sum_J c_aJ L~_Ji  ([K][vec][ai]),
  // G[ai][vec, bj] = sum_K L~^K_ai dL~^K_bj
  // (the effective MLCC2 transformation works per occupied-pair block instead)
  const bool eff_blocks = model == MLCC_MLCC2 && !has_c2 && std::isfinite(w_eff);
  dLai.ensure(al, (size_t)J * b * M * sizeof(T));
  if (!eff_blocks) Gm.ensure(al, (size_t)M * b * M * sizeof(double));
  // one launch per term: rows (K, a) x columns (vec, i), then rows (vec, a) x
  // columns (K, i) (MLCC2: K the low part of the two-level index)
  if (model == MLCC_MLCC2) {
    // pair-major dL~: dLai[vec][ai][K]; K is the low part of the two-level
    // output index, so the output rows / columns of a tile are contiguous
    G(J * v, b * o, V).A(lt + O * n + O, n2, 1).Mhi(J, n, o * J).B(ctt, 1, V).Nhi(o, n1, M * J)
        .C(dLai.p, 1, J).tag("dLai").run(x, p, o64);
    G(b * v, J * o, O).A(ct, O, 1).Mhi(v, n1, M * J).B(loot, 1, O * O).Nhi(J, O, J)
        .C(dLai.p, o * J, 1, 0, -1.0, 1.0).tag("dLai").run(x, p, o64);
    if (!eff_blocks)
      G(M, b * M, J).A(off<T>(LaiT), J, 1).B(dLai.p, 1, J).C(Gm.p, b * M, 1)
          .tag("sigma2_LdL").run(x, p, true);
  } else {
    // K-major dL~: dLai[K][vec][ai] (read so by the MLCCSD doubles terms)
    G(J * v, b * o, V).A(lt + O * n + O, n, 1).Mhi(v, n2, b * M).B(ct, O, 1).Nhi(o, n1, M)
        .C(dLai.p, o, 1).tag("dLai").run(x, p, o64);
    G(b * v, J * o, O).A(ct, O, 1).Mhi(v, n1, M).B(lt, n, 1).Nhi(o, n2, b * M)
        .C(dLai.p, o, 1, 0, -1.0, 1.0).tag("dLai").run(x, p, o64);
    G(M, b * M, J).A(off<T>(Lai), 1, M).B(dLai.p, b * M, 1).C(Gm.p, b * M, 1)
        .tag("sigma2_LdL").run(x, p, true);
  }

  Zc.ensure(al, (size_t)(J + 1) * b * M * sizeof(T));
  if (eff_blocks) {
    eff_doubles_pairblocks_t<T>(nb, w_eff);
  } else {
    full_doubles_to_singles_t<T>(nb, c, ld, has_c2, sigma, w_eff);
    if (!has_c2 && !std::isfinite(w_eff)) return;
  }
  // sigma_AI += sum_Kb L~^K_Ab Zc^K_bi  (A1-type)  - sum_Kk L~^K_kI Zc^K_ak  (B1-type)
  G(V, b * o, v, J).A(lt + O * n + O, n, 1, n2).B(Zc.p, 1, v, b * M).Nhi(o, M, ld)
      .C(sigma, O, 1, 0, 1.0, 1.0).tag("d2s_A1").run(x, p, true);
  G(O, v, o, J, b).A(lt, 1, n, n2, 0).B(Zc.p, v, 1, b * M, M).C(sigma, 1, O, ld, -1.0, 1.0)
      .tag("d2s_B1").run(x, p, true);
  // sigma_ai += sum_bj u_aibj F~_jb  (row J of Zc)
  k::acc3d<T>(x, b, v, o, 1.0, off<T>(Zc, J * b * M), M, 1, v, sigma, ld, O);
}

// Effective transformation (MLCC2): c2 = P[L~ dL~] / (w - eps) per
// occupied-pair block (I, J), I <= J, for the nb vectors at once (dL~ is
// pair-major, dLai[vec][ai][K]):
//   off-diagonal  X = L~_I^T dL~_J, then X = (dL~_I^T L~_J + X) / (w - eps)
//                 (FP64 denominator in the GEMM epilogue)
//   diagonal      X = L~_I^T dL~_I, Y = (X + X^T) / (w - eps)
// then u(c2) of the block and its mirror, Zc_I += L_J u_IJ^T and
// Zc_J += L_I u_JI^T.  Zc[K][vec][i][a] (K = J: the F~_jb row).
template <typename T> void mlcc_problem::eff_doubles_pairblocks_t(int nb, double w) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t J = d.J, M = d.M, o = d.o, v = d.v, b = nb;
  const Prec p = gemm_prec<T>();
  const int ob = occ_batch(nb);
  const int64_t Rm = (int64_t)std::min<int64_t>(ob, o) * v;
  pbX.ensure(al, (size_t)b * Rm * Rm * sizeof(double));
  pbY.ensure(al, (size_t)b * Rm * Rm * sizeof(double));
  pbU1.ensure(al, (size_t)b * Rm * Rm * sizeof(T));
  pbU2.ensure(al, (size_t)b * Rm * Rm * sizeof(T));
  MLCC_HIP(hipMemsetAsync(Zc.p, 0, (size_t)(J + 1) * b * M * sizeof(T), x.stream));
  // F~_jb (occupied-major) in the spare row of LvoJ: row J of Zc is sum_bj u_aibj F~_jb
  k::pack2d<T, double>(x, off<T>(LvoJ, J * M), Ft.as<double>() + d.O, 1, 0, o, v, d.n);
  const T *lai = off<T>(LaiT), *dl = off<T>(dLai);
  const double *eT = eps_aiT.as<double>();
  for (int i0 = 0; i0 < o; i0 += ob) {
    const int ni = (int)std::min<int64_t>(ob, o - i0);
    const int64_t RI = (int64_t)ni * v;
    for (int j0 = i0; j0 < o; j0 += ob) {
      const int nj = (int)std::min<int64_t>(ob, o - j0);
      const int64_t RJ = (int64_t)nj * v, blk = RI * RJ;
      const bool diag = j0 == i0;
      const double *xv;
      G(RI, RJ, J, 1, b).A(lai + i0 * J, o * J, 1, 0, 0).Mhi(v, J, v * RJ)
          .B(dl + j0 * J, 1, o * J, 0, M * J).Nhi(v, J, v).C(pbX.p, RJ, 1, blk)
          .tag("sigma2_LdL").run(x, p, true);
      if (diag) {
        k::sym_div<double, double>(x, RI, pbX.as<double>(), RI, eT + i0 * v, w,
                                   pbY.as<double>(), (int)b, blk, blk);
        xv = pbY.as<double>();
      } else {
        G(RI, RJ, J, 1, b).A(dl + i0 * J, o * J, 1, 0, M * J).Mhi(v, J, v * RJ)
            .B(lai + j0 * J, 1, o * J, 0, 0).Nhi(v, J, v).C(pbX.p, RJ, 1, blk, -1.0, -1.0)
            .den(eT + i0 * v, eT + j0 * v, -w).tag("sigma2_LdL").run(x, p, true);
        xv = pbX.as<double>();
      }
      k::u_pairblock<T>(x, (int)o, (int)v, ni, nj, xv, RJ, blk, off<T>(pbU1), RJ,
                        diag ? nullptr : off<T>(pbU2), RI, blk, (int)b, nullptr, i0, j0);
      G(J + 1, RI, RJ, 1, b).A(off<T>(LvoJ, j0 * v), M, 1, 0, 0).B(pbU1.p, 1, RJ, 0, blk)
          .C(off<T>(Zc, i0 * v), b * M, 1, M, 1.0, 1.0).tag("Zc_uL").run(x, p, sizeof(T) == 8);
      if (!diag)
        G(J + 1, RJ, RI, 1, b).A(off<T>(LvoJ, i0 * v), M, 1, 0, 0).B(pbU2.p, 1, RI, 0, blk)
            .C(off<T>(Zc, j0 * v), b * M, 1, M, 1.0, 1.0).tag("Zc_uL")
            .run(x, p, sizeof(T) == 8);
    }
  }
}

// Doubles -> singles of the full-space transformation (trial doubles) and of
// the effective one on the stored-doubles path: c2 into u(c2) and Zc.
template <typename T>
void mlcc_problem::full_doubles_to_singles_t(int nb, const double *c, int64_t ld, bool has_c2,
                                            double *sigma, double w_eff) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t J = d.J, n = d.n, O = d.O, M = d.M, n1 = d.n1, b = nb;
  const Prec p = gemm_prec<T>();
  const bool o64 = sizeof(T) == 8;
  const double *F = Ft.as<double>();
  // the doubles used by doubles -> singles: the trial doubles, or the
  // eliminated ones of the effective transformation
  const double *c2base = nullptr;
  int64_t c2ld = 0;
  if (has_c2) {
    c2base = c + n1;
    c2ld = ld;
    if (model == MLCC_MLCC2) {
      k::sym_plus_diag<double>(x, M, Gm.as<double>(), b * M, eps_ai.as<double>(), c + n1,
                               sigma + n1, (int)b, M, ld, ld);
    } else {
      for (int64_t vec = 0; vec < b; ++vec)
        ccsd_sigma2_t<T>(c + vec * ld, c + vec * ld + n1, Gm.as<double>() + vec * M, b * M,
                         off<T>(dLai, vec * M), b * M, sigma + vec * ld + n1);
    }
  } else if (std::isfinite(w_eff)) {
    c2e.ensure(al, (size_t)b * M * M * sizeof(double));
    k::sym_div<double, double>(x, M, Gm.as<double>(), b * M, eps_ai.as<double>(), w_eff,
                               c2e.as<double>(), (int)b, M, M * M);
    c2base = c2e.as<double>();
    c2ld = M * M;
  }
  if (!c2base) return;
  // doubles -> singles: the Omega_1 doubles terms with u = 2 c2 - c2(i<->j).
  // The rows of u(c2) are stored occupied-major (row (c,j) at j*v + c), so
  // Zc^K[vec][j][c] = sum_bk L_bk^K u_cj,bk has c contiguous, the reduction
  // index of the A1 term.
  ut.ensure(al, (size_t)b * M * M * sizeof(T));
  k::u_of<T>(x, d.o, d.v, c2base, off<T>(ut), (int)b, c2ld, M * M, true);
  // F~_jb in the spare row J of L_vo: row J of Zc is sum_bj u_aibj F~_jb
  k::pack2d_t<T, double>(x, off<T>(Lvo0, J * M), F + O, 1, 0, d.o, d.v, n);
  G(J + 1, b * M, M).A(off<T>(Lvo0), M, 1).B(ut.p, 1, M).Nhi(M, M * M, M).C(Zc.p, b * M, 1)
      .tag("Zc_uL").run(x, p, o64);
}

static constexpr int kMaxBatch = 8;

// Trial vectors per batch: up to 8, fewer when the per-vector scratch of a
// batch would pass 48 GB: W (J V O), dL~ and Zc (about 2 J M) and P (J o O)
// in the operand type, and on the stored-doubles path G in FP64, the
// eliminated doubles in FP64 and u(c2) in the operand type (M*M each).
int mlcc_problem::max_batch(bool eff) const {
  const double ts = (double)tsize;
  const double per = ts * ((double)d.J * d.V * d.O + 2.0 * (double)d.J * d.M +
                           (double)d.J * d.o * d.O);
  double cap = std::floor(48e9 / per);
  if (has_doubles() && !(eff && model == MLCC_MLCC2))
    cap = std::min(cap, std::floor(48e9 / ((double)d.M * (double)d.M * (16.0 + ts))));
  return (int)std::max(1.0, std::min((double)kMaxBatch, cap));
}

void mlcc_problem::transform(int nvec, const double *c, double *sigma) {
  const int64_t dm = dim();
  const int mb = max_batch(false);
  for (int i0 = 0; i0 < nvec; i0 += mb) {
    const int nb = std::min(mb, nvec - i0);
    if (prec == MLCC_FP64)
      transform_batch_t<double>(nb, c + i0 * dm, dm, has_doubles(), sigma + i0 * dm, NAN);
    else
      transform_batch_t<float>(nb, c + i0 * dm, dm, has_doubles(), sigma + i0 * dm, NAN);
  }
}

void mlcc_problem::transform_eff(double w, int nvec, const double *c1, double *s1) {
  const int mb = max_batch(true);
  for (int i0 = 0; i0 < nvec; i0 += mb) {
    const int nb = std::min(mb, nvec - i0);
    if (prec == MLCC_FP64)
      transform_batch_t<double>(nb, c1 + i0 * d.n1, d.n1, false, s1 + i0 * d.n1, w);
    else
      transform_batch_t<float>(nb, c1 + i0 * d.n1, d.n1, false, s1 + i0 * d.n1, w);
  }
}
