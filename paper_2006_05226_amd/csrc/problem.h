// The context and problem objects behind the C ABI.
#pragma once

#include <atomic>
#include <memory>
#include <string>

#include "mlcc_internal.h"

struct mlcc_context {
  // contractions that run plain BF16 products in MLCC_BF16 (mlcc_bf16_map)
  std::vector<std::string> bf16_map;
  // references: the creator's, one per problem created on it and one per
  // server; the context is freed when the last one is dropped, so that
  // destroying it before its problems is safe
  std::atomic<int> refs{1};
  int device = 0;
  mlcc::Profiler prof;
  bool own_stream = false;
  mlcc::Alloc al;
  mlcc::Exec ex;
  int pair_occ = 0;  // forced occupied indices per pair block (0: memory rule)
  std::string last_error;
  std::mutex err_mu;
};

namespace mlcc {

// Drops one reference on a context; the last one frees it.
void context_unref(mlcc_context *ctx);

struct Dims {
  int O = 0, V = 0, n = 0, J = 0, o = 0, v = 0;
  // CCSD space of three-level MLCCSD (prefixes of the active space); equal to
  // (o, v) for the other models
  int ot = 0, vt = 0;
  int64_t M = 0, n1 = 0, n2 = 0;  // pairs, singles, n*n
  int64_t dim_full() const { return n1 + M * M; }
  // some active doubles are projected at the CC2 level (three-level MLCCSD)
  bool cc2_rows() const { return ot < o || vt < v; }
};

// Builder for one GEMM-engine call.
struct G {
  GemmArgs a;
  G(int64_t M, int64_t N, int64_t K, int64_t R = 1, int64_t Z = 1) {
    a.M = M; a.N = N; a.K = K; a.R = R; a.Z = Z;
  }
  G &A(const void *p, int64_t sm, int64_t sk, int64_t sr = 0, int64_t sz = 0) {
    a.A = p; a.sAm = sm; a.sAk = sk; a.sAr = sr; a.sAz = sz;
    return *this;
  }
  G &B(const void *p, int64_t sk, int64_t sn, int64_t sr = 0, int64_t sz = 0) {
    a.B = p; a.sBk = sk; a.sBn = sn; a.sBr = sr; a.sBz = sz;
    return *this;
  }
  G &C(void *p, int64_t sm, int64_t sn, int64_t sz = 0, double alpha = 1.0, double beta = 0.0,
       const void *cin = nullptr) {
    a.C = p; a.sCm = sm; a.sCn = sn; a.sCz = sz; a.alpha = alpha; a.beta = beta;
    a.Cin = cin ? cin : p;
    return *this;
  }
  // two-level rows: m = (hi, lo) with lo < mlo; strides of hi for A and C
  G &Mhi(int64_t mlo, int64_t sA_hi, int64_t sC_hi) {
    a.Mlo = mlo; a.sAm_hi = sA_hi; a.sCm_hi = sC_hi;
    return *this;
  }
  // two-level columns: n = (hi, lo) with lo < nlo; strides of hi for B and C
  G &Nhi(int64_t nlo, int64_t sB_hi, int64_t sC_hi) {
    a.Nlo = nlo; a.sBn_hi = sB_hi; a.sCn_hi = sC_hi;
    return *this;
  }
  G &tag(const char *t) {
    a.tag = t;
    return *this;
  }
  // epilogue denominator: C = (alpha acc + beta Cin) / (row[m] + col[n] + shift)
  G &den(const double *row, const double *col, double shift = 0.0) {
    a.den_row = row; a.den_col = col; a.den_shift = shift;
    return *this;
  }
  void run(Exec &ex, Prec p, bool out64) const { gemm(ex, p, a, out64); }
};

template <typename T> inline Prec prec_of() { return sizeof(T) == 8 ? Prec::F64 : Prec::F32; }

// Bytes of the pair-block buffers of the MLCC2 doubles, and the occupied
// indices per block that keep nz blocks within them (operand size tsize).
constexpr double kPairBlockBytes = 4e9;
int pair_block_occ(int o, int v, int nz, int tsize);
template <typename T> inline T *off(const DBuf &b, int64_t elems = 0) {
  return static_cast<T *>(b.p) + elems;
}
template <typename T> inline T *off(void *p, int64_t elems) { return static_cast<T *>(p) + elems; }
template <typename T> inline const T *off(const void *p, int64_t elems) {
  return static_cast<const T *>(p) + elems;
}

}  // namespace mlcc

namespace mlcc {
struct CcsdState;  // MLCCSD doubles: integral blocks, intermediates (ccsd.inl)
}

struct mlcc_problem {
  ~mlcc_problem();
  mlcc::CcsdState *cc = nullptr;
  mlcc_context *ctx = nullptr;
  mlcc::Exec *ex = nullptr;
  mlcc::Dims d;
  int model = MLCC_MLCC2;
  int prec = MLCC_FP64;
  size_t tsize = 8;  // bytes of the operand type

  // inputs and derived constants
  mlcc::DBuf L, eps, h, eps_ai, eps_vo, Lvo0;
  mlcc::DBuf eps_aiT;  // f64 [o][v]: e_a - e_i in occupied-major pair order (i v + a)
  mlcc::DBuf LvoJ;     // op [J+1][o][v]: L^K_bj occupied-major (row J: F~_jb)
  mlcc::DBuf fock;     // f64 [n][n] when the desc gave a Fock matrix (else diag(eps))
  // state at the current amplitudes
  mlcc::DBuf amp;      // f64 [n1 (+ M*M for MLCCSD)]: t1 then the MLCCSD doubles
  mlcc::DBuf s2, o2;   // MLCC2, on demand: f64 [M][M] doubles and doubles residual
  mlcc::DBuf t1T;      // op [n1]
  mlcc::DBuf Lt, ht, Ft, dK, dKT;
  mlcc::DBuf Lai, LaiT, g, u, Z;
  mlcc::DBuf om;       // f64 [n1 + M*M]
  mlcc::DBuf res;      // f64 device scalars
  // Jacobian intermediates
  mlcc::DBuf Xint, Yint, fvec, LooT;
  // MLCCSD intermediates and scratch
  mlcc::DBuf cc_work;
  // transform scratch
  mlcc::DBuf cT, cTt, Xk, W, P, qv, rv, wv, ut, Zc, dLai, Gm, c2e;
  // occupied-pair blocks of the MLCC2 doubles (ground state with analytic s2,
  // effective transformation): f64 values and u in the operand type
  mlcc::DBuf pbX, pbY, pbU1, pbU2;

  bool have_amp = false;
  bool x2_set = false;     // MLCC2: an independent s2 was given
  bool state_valid = false;  // dressed quantities match amp
  bool jac_ready = false;
  bool fock_full = false;
  bool u_occ = false;      // u is stored in occupied-major pair order, rows and columns
  bool want_s = false;     // the next state evaluation also writes the analytic s2
  bool want_om2 = false;   // ... and the MLCC2 doubles residual
  double e_corr = 0.0;
  double omega_norm = 0.0;

  bool has_doubles() const { return model != MLCC_CCS && d.M > 0; }
  int64_t dim() const { return d.n1 + (has_doubles() ? d.M * d.M : 0); }
  int max_batch(bool eff) const;  // trial vectors per Jacobian batch
  // contraction precision for operand type T (FP32 storage may run split
  // BF16 products)
  template <typename T> mlcc::Prec gemm_prec() const {
    return sizeof(T) == 8 ? mlcc::Prec::F64
                          : prec == MLCC_BF16X3 ? mlcc::Prec::BF16X3
                          : prec == MLCC_BF16   ? mlcc::Prec::BF16
                                                : mlcc::Prec::F32;
  }
  double *t1() const { return amp.as<double>(); }
  // doubles amplitudes and residual: MLCCSD t2 after t1; MLCC2 s2 in its own
  // array, allocated on demand (ensure_doubles)
  double *x2() const {
    return model == MLCC_MLCCSD ? amp.as<double>() + d.n1 : s2.as<double>();
  }
  double *om2() const {
    return model == MLCC_MLCCSD ? om.as<double>() + d.n1 : o2.as<double>();
  }
  void ensure_doubles() {
    if (model == MLCC_MLCC2 && d.M > 0) {
      s2.ensure(ex->al, (size_t)d.M * d.M * sizeof(double));
      o2.ensure(ex->al, (size_t)d.M * d.M * sizeof(double));
    }
  }
  // occupied indices per block of the pair-blocked doubles, for nz vectors
  int occ_batch(int nz) const;

  // model steps (problem.cpp)
  void setup(const mlcc_problem_desc &desc);
  // dress + doubles + Z + Omega + energy; keep_u: store the ground-state u
  // (the Jacobian's singles terms read it)
  void compute_state(bool full_fock, bool keep_u = false);
  void prepare_jacobian();
  void transform(int nvec, const double *c, double *sigma);       // device pointers
  void transform_eff(double w, int nvec, const double *c1, double *s1);
  double fetch(const double *dev);
  void fetch_n(const double *dev, double *host, int n);
  // CNTOs from excitation vectors (cnto.cpp); R [ns][V][O] device, w [ns] host
  void cnto(int ns, const double *R, const double *w, int o_act, int v_act, double *m_eig,
            double *n_eig, double *C, double *eps_out, double *fock_out, double *L_out,
            bool L_out_dev);

 private:
  template <typename T> void setup_t(const double *Lhost_or_dev, bool dev,
                                     const uint64_t *synth_seed);
  template <typename T> void dress_t(bool full_fock);
  template <typename T> void doubles_mlcc2_t();
  template <typename T> void doubles_pairblocks_t(bool keep_u);
  template <typename T> void eff_doubles_pairblocks_t(int nb, double w);
  template <typename T> void omega_singles_t(const void *Zb, const void *ub, double *om1,
                                             bool add_fock);
  template <typename T> void compute_state_t(bool full_fock, bool keep_u);
  template <typename T> void prepare_jacobian_t();
  template <typename T> void transform_batch_t(int nb, const double *c, int64_t ld,
                                               bool has_c2, double *sigma, double w_eff);
  template <typename T> void full_doubles_to_singles_t(int nb, const double *c, int64_t ld,
                                                       bool has_c2, double *sigma,
                                                       double w_eff);
  template <typename T> void cnto_t(int ns, const double *R, const double *w, int o_act, int v_act,
                                    double *m_eig, double *n_eig, double *C, double *eps_out,
                                    double *fock_out, double *L_out, bool L_out_dev);
  template <typename T> void ccsd_integrals_t();
  template <typename T> void ccsd_omega2_t();
  template <typename T> void ccsd_prepare_t();
  // MLCCSD doubles of sigma for one vector; Gv[ai][bj] (row stride ldg) holds
  // sum_K L~^K_ai dL~^K_bj and dLvo[K][ai] (row stride ldl) the derivative
  // dL~_ai of that vector
  template <typename T> void ccsd_sigma2_t(const double *c1, const double *c2, const double *Gv,
                                           int64_t ldg, const void *dLvo, int64_t ldl,
                                           double *s2);
  template <typename T> void ccsd_terms_t(const void *const *blk, const void *tA, const void *uA,
                                          const void *tB, const void *uB, bool incL, bool incB,
                                          bool incQ, bool ladder, double *sym, double *R);
};
