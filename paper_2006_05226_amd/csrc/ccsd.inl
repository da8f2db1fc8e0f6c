// MLCCSD (CCS/CCSD) doubles: the Omega_2 residual and the doubles part of the
// Jacobian transformation (included by problem.cpp).
//
// Omega_2 is the closed-shell CCSD doubles residual with X1-dressed integrals
// and every explicit index in the active space (Sec. 2.1 eq. mlccsd_2;
// Appendix A.1, MLCCSD Omega vector, in the standard spin-adapted form):
//
//   Omega = A2 + B2 + P(C2 + D2 + E2),   P X_aibj = X_aibj + X_bjai
//   A2 = g_aibj + sum_cd t_cidj g_acbd                          (ladder)
//   B2 = sum_kl t_akbl (g_kilj + sum_cd t_cidj g_kcld)
//   C2 = -1/2 sum_ck t_bkcj Y_aick - sum_ck t_bkci Y_ajck,
//        Y_aick = g_kiac - 1/2 sum_dl t_aldi g_kdlc
//   D2 = 1/2 sum_ck u_bjck (L_aikc + 1/2 sum_dl u_aidl L_ldkc)
//   E2 = sum_c t_aicj (F_bc - sum_dkl u_bkdl g_ldkc)
//        - sum_k t_aibk (F_kj + sum_cdl u_cldj g_kdlc)
//
// The residual is evaluated by one routine in "slot" form: every term holds
// exactly one integral (or Fock) factor and at most two amplitude factors,
// the first from slot A and the second from slot B.  The Jacobian doubles
// (Appendix A.2, the derivative of Omega_2) are then three evaluations:
//   (dg, dF; t, t) + (g, F; dt, t)[terms with t] + (g, F; t, dt)[terms with t t]
// with dL~ = L~ C - C L~ (C[A][I] = c_AI) giving the dressed-integral
// derivatives.  Every term with two amplitudes contains g_ovov, whose
// derivative vanishes (the ov block of L~ does not depend on t1).  The ladder
// integral derivative is taken through Y3_Kibj = sum_cd g_Kcbd t_cidj so that
// the v^4 integrals are never differentiated per vector.
//
// All contractions are GEMM-engine calls; two-level row/column indices and
// the batch-reduce index let one call regroup 4-index tensors (e.g. the
// ladder contracts (c, d) as (r, k) with rows (a, b) and columns (i, j)).
// Doubles arrays are [M][M] with pair index a*o + i: strides a: o*M, i: M,
// b: o, j: 1.
//
// Three-level MLCCSD (CCS/CC2/CCSD) uses the same terms with their output
// restricted to the CCSD space (a, b < vt; i, j < ot) while every summation
// index runs over the whole active space: the output row and column counts
// of each call shrink (rows (a, i) become two-level (a < vt, i < ot); terms
// over three output indices take the leading one as a batch index), and the
// ladder integrals are kept only for a, b < vt, g_vvvv[(a,c)][(b,d)] with
// leading dimension vt*v.  The remaining entries are then overwritten with
// their CC2-level values g~ + eps x (k::cc2_rows).

namespace mlcc {
struct CcsdState {
  DBuf Loo, Lvv, LKc, Lkc;                        // packed L~ blocks [J][..]
  DBuf g_vovo, g_oooo, g_ovov, g_oovv, g_voov;    // integral blocks (op type)
  DBuf gX;                                        // gX[(c,k)][(d,l)] = g_kdlc
  DBuf xA, xB;                                    // occupied-exchanged amplitudes
  DBuf tL;                                        // tL[c][i][j][d] = t_cidj (slot A)
  DBuf g_vvvv;                                    // [(a,c)][(b,d)]
  DBuf Fvv, Foo;                                  // dressed Fock blocks (op type)
  DBuf tT;                                        // t2 in the op type
  DBuf Q, Y, Z, X, Rb, Lld, g2, g3, Wvv, Woo;     // term scratch
  DBuf Gk, Y3;                                    // ladder-derivative intermediate
  // per-vector Jacobian scratch
  DBuf c1T, c1tt, c2T, cu2, dLoo, dLvv, dg_oooo, dg_oovv, dg_voov, dF64, dFvv, dFoo, dXk, Pv, Po;
  DBuf S, Rs;
};
}  // namespace mlcc

mlcc_problem::~mlcc_problem() { delete cc; }

// Integral blocks of the active space from the current L~ and F~.
template <typename T> void mlcc_problem::ccsd_integrals_t() {
  Exec &x = *ex;
  Alloc *al = ex->al;
  if (!cc) cc = new CcsdState();
  CcsdState &s = *cc;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O, o = d.o, v = d.v, M = d.M;
  const Prec p = gemm_prec<T>();
  const bool o64 = sizeof(T) == 8;
  const T *lt = off<T>(Lt);
  s.Loo.ensure(al, J * o * o * sizeof(T));
  s.Lvv.ensure(al, J * v * v * sizeof(T));
  k::pack2d<T, T>(x, off<T>(s.Loo), lt, J, n2, o, o, n);
  k::pack2d<T, T>(x, off<T>(s.Lvv), lt + O * n + O, J, n2, v, v, n);
  // Lai (L~_ai) is packed already; Lkc[J][k][c] = L~_kc = L_kc (the ov block
  // does not depend on t1) with the pair index k*v + c contiguous
  const T *Lvo = off<T>(Lai);
  s.Lkc.ensure(al, J * o * v * sizeof(T));
  k::pack2d<T, T>(x, off<T>(s.Lkc), lt + O, J, n2, o, v, n);
  s.g_vovo.ensure(al, M * M * sizeof(T));
  s.g_oooo.ensure(al, o * o * o * o * sizeof(T));
  s.g_ovov.ensure(al, M * M * sizeof(T));
  s.g_oovv.ensure(al, o * o * v * v * sizeof(T));
  s.g_voov.ensure(al, M * M * sizeof(T));
  const int64_t vt = d.vt;
  s.g_vvvv.ensure(al, vt * v * vt * v * sizeof(T));
  G(M, M, J).A(Lvo, 1, M).B(Lvo, M, 1).C(s.g_vovo.p, M, 1).tag("cc_g").run(x, p, o64);
  G(o * o, o * o, J).A(s.Loo.p, 1, o * o).B(s.Loo.p, o * o, 1).C(s.g_oooo.p, o * o, 1)
      .tag("cc_g").run(x, p, o64);
  // g_ovov[(k,c)][(l,d)] = g_kcld
  G(M, M, J).A(s.Lkc.p, 1, M).B(s.Lkc.p, M, 1).C(s.g_ovov.p, M, 1).tag("cc_g").run(x, p, o64);
  G(o * o, v * v, J).A(s.Loo.p, 1, o * o).B(s.Lvv.p, v * v, 1).C(s.g_oovv.p, v * v, 1)
      .tag("cc_g").run(x, p, o64);
  G(M, M, J).A(Lvo, 1, M).B(s.Lkc.p, M, 1).C(s.g_voov.p, M, 1).tag("cc_g").run(x, p, o64);
  // g_vvvv[(a,c)][(b,d)] = g~_acbd for a, b in the CCSD space (a prefix of the pair order)
  G(vt * v, vt * v, J).A(s.Lvv.p, 1, v * v).B(s.Lvv.p, v * v, 1).C(s.g_vvvv.p, vt * v, 1)
      .tag("cc_g_vvvv").run(x, p, o64);
  // gX[(c,k)][(d,l)] = g_kdlc = g_ovov[(k,d)][(l,c)], the C2 integral with
  // its reduction pair (d,l) contiguous (symmetric under (c,k) <-> (d,l))
  s.gX.ensure(al, M * M * sizeof(T));
  {
    const int64_t nn[4] = {v, o, v, o}, ss[4] = {1, v * M, M, v};
    k::permute4<T, T>(x, off<T>(s.gX), off<T>(s.g_ovov), nn, ss, 1.0, 0.0);
  }
  s.Fvv.ensure(al, v * v * sizeof(T));
  s.Foo.ensure(al, o * o * sizeof(T));
  k::pack2d<T, double>(x, off<T>(s.Fvv), Ft.as<double>() + O * n + O, 1, 0, v, v, n);
  k::pack2d<T, double>(x, off<T>(s.Foo), Ft.as<double>(), 1, 0, o, o, n);
}

// Block table passed to ccsd_terms_t: vovo, oooo, ovov, oovv, voov, vvvv, Fvv, Foo
enum { CB_VOVO, CB_OOOO, CB_OVOV, CB_OOVV, CB_VOOV, CB_VVVV, CB_FVV, CB_FOO, CB_N };

// sym += A2 + B2 (symmetric by themselves), R += C2 + D2 + E2.  Slot A feeds
// the terms with one amplitude and the first amplitude of the others; slot B
// the second.  incL/incB/incQ select the terms with zero/one/two amplitudes;
// ladder adds sum_cd tA_cidj g_acbd.  A null ovov block means g_ovov = 0.
template <typename T>
void mlcc_problem::ccsd_terms_t(const void *const *blk, const void *tA, const void *uA,
                                const void *tB, const void *uB, bool incL, bool incB, bool incQ,
                                bool ladder, double *sym, double *R) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  CcsdState &s = *cc;
  const int64_t o = d.o, v = d.v, M = d.M, ot = d.ot, vt = d.vt, Mt = ot * vt;
  const bool full = !d.cc2_rows();  // output over the whole active space
  const Prec p = gemm_prec<T>();
  const bool o64 = sizeof(T) == 8;
  if (!blk[CB_OVOV]) incQ = false;
  const bool any = incB || incQ;
  // --- A2
  if (incL) {
    const int64_t nn[4] = {1, 1, M, M}, ss[4] = {0, 0, M, 1};
    k::permute4<double, T>(x, sym, static_cast<const T *>(blk[CB_VOVO]), nn, ss, 1.0, 1.0);
  }
  if (Mt == 0) return;  // no CCSD-level projection
  // tL[c][i][j][d] = tA_cidj: the ladder and E2 reduce over its contiguous d
  if ((ladder && incB) || any) {
    const int64_t nn[4] = {v, o, o, v}, sl[4] = {o * M, M, 1, o};
    s.tL.ensure(al, M * M * sizeof(T));
    k::permute4<T, T>(x, off<T>(s.tL), static_cast<const T *>(tA), nn, sl, 1.0, 0.0);
  }
  if (ladder && incB) {
    G(vt * vt, ot * ot, v, v).A(blk[CB_VVVV], v, 1, vt * v).Mhi(vt, v * vt * v, o * M)
        .B(s.tL.p, 1, v, o * o * v).Nhi(ot, o * v, M).C(sym, o, 1, 0, 1.0, 1.0)
        .tag("cc_ladder").run(x, p, true);
  }
  if (!any) return;
  // --- B2: Q[k][l][i][j] = g_kilj + sum_cd tB_cidj g_kcld ; sym += sum_kl tA_akbl Q_klij
  s.Q.ensure(al, o * o * o * o * sizeof(T));
  {
    const int64_t nn[4] = {o, o, o, o}, ss[4] = {o * o * o, o, o * o, 1};
    k::permute4<T, T>(x, off<T>(s.Q), static_cast<const T *>(blk[CB_OOOO]), nn, ss,
                      incB ? 1.0 : 0.0, 0.0);
  }
  if (incQ)
    G(o * o, ot * ot, v, v).A(blk[CB_OVOV], v, 1, M).Mhi(o, v * M, o * o * o)
        .B(tB, o, 1, o * M).Nhi(ot, M, o).C(s.Q.p, o * o, 1, 0, 1.0, 1.0).tag("cc_B2")
        .run(x, p, o64);
  G(vt * vt, ot * ot, o, o).A(tA, o, 1, M).Mhi(vt, o * M, o * M).B(s.Q.p, o * o, 1, o * o * o)
      .Nhi(ot, o, M).C(sym, o, 1, 0, 1.0, 1.0).tag("cc_B2").run(x, p, true);
  // --- C2: Y[(a,i)][(c,k)] = g_kiac - 1/2 sum_dl tB_aldi g_kdlc ;
  //         X[(a,i)][(b,j)] = sum_ck Y[(a,i)][(c,k)] tA_bkcj ; R += -1/2 X - X(i<->j)
  // Both sums run over one contiguous pair index through the occupied-
  // exchanged amplitudes x[(a,i)][(b,j)] = t_ajbi: tB_aldi = xB[(a,i)][(d,l)],
  // tA_bkcj = xA[(b,j)][(c,k)].
  s.Y.ensure(al, M * M * sizeof(T));
  s.X.ensure(al, M * M * sizeof(double));
  {
    const int64_t nn[4] = {v, o, v, o}, ss[4] = {v, v * v, 1, o * v * v};
    k::permute4<T, T>(x, off<T>(s.Y), static_cast<const T *>(blk[CB_OOVV]), nn, ss,
                      incB ? 1.0 : 0.0, 0.0);
  }
  {
    const int64_t nn[4] = {v, o, v, o}, sx[4] = {o * M, 1, o, M};
    s.xA.ensure(al, M * M * sizeof(T));
    k::permute4<T, T>(x, off<T>(s.xA), static_cast<const T *>(tA), nn, sx, 1.0, 0.0);
    if (incQ) {
      MLCC_REQUIRE(blk[CB_OVOV] == s.g_ovov.p, MLCC_E_STATE, "C2: gX belongs to g_ovov");
      const void *xB = s.xA.p;
      if (tB != tA) {
        s.xB.ensure(al, M * M * sizeof(T));
        k::permute4<T, T>(x, off<T>(s.xB), static_cast<const T *>(tB), nn, sx, 1.0, 0.0);
        xB = s.xB.p;
      }
      // rows (a, i) of the CCSD space: two-level (a, i < ot)
      G(Mt, M, M).A(xB, M, 1).Mhi(ot, o * M, o * M).B(s.gX.p, 1, M)
          .C(s.Y.p, M, 1, 0, -0.5, 1.0).tag("cc_C2").run(x, p, o64);
    }
  }
  if (!full) k::fill(x, s.X.as<double>(), M * M, 0.0);
  G(Mt, Mt, M).A(s.Y.p, M, 1).Mhi(ot, o * M, o * M).B(s.xA.p, 1, M).Nhi(ot, o * M, o)
      .C(s.X.p, M, 1).tag("cc_C2").run(x, p, true);
  {
    const int64_t nn[4] = {v, o, v, o};
    const int64_t sx[4] = {o * M, 1, o, M}, sid[4] = {o * M, M, o, 1};
    k::permute4<double, double>(x, R, s.X.as<double>(), nn, sx, -1.0, 1.0);
    k::permute4<double, double>(x, R, s.X.as<double>(), nn, sid, -0.5, 1.0);
  }
  // --- D2: Z[(a,i)][(c,k)] = L_aikc + 1/2 sum_dl uB_aidl L_ldkc ; R += 1/2 Z uA
  // (Lld and uA are symmetric under the exchange of their pair indices, so
  // both are read with the reduction pair contiguous)
  s.Z.ensure(al, M * M * sizeof(T));
  {
    const int64_t nn[4] = {v, o, v, o};
    const int64_t s1[4] = {o * M, M, 1, v};          // g_aikc from g_voov[(a,i)][(k,c)]
    const int64_t s2[4] = {v, v * v, 1, o * v * v};  // g_acki from g_oovv[(k,i)][(a,c)]
    k::permute4<T, T>(x, off<T>(s.Z), static_cast<const T *>(blk[CB_VOOV]), nn, s1,
                      incB ? 2.0 : 0.0, 0.0);
    k::permute4<T, T>(x, off<T>(s.Z), static_cast<const T *>(blk[CB_OOVV]), nn, s2,
                      incB ? -1.0 : 0.0, 1.0);
  }
  if (incQ) {
    s.Lld.ensure(al, M * M * sizeof(T));
    const int64_t nn[4] = {v, o, v, o};                  // Lld[d][l][c][k] = L_ldkc
    const int64_t s1[4] = {M, v * M, 1, v}, s2[4] = {1, v * M, M, v};
    k::permute4<T, T>(x, off<T>(s.Lld), static_cast<const T *>(blk[CB_OVOV]), nn, s1, 2.0, 0.0);
    k::permute4<T, T>(x, off<T>(s.Lld), static_cast<const T *>(blk[CB_OVOV]), nn, s2, -1.0, 1.0);
    G(Mt, M, M).A(uB, M, 1).Mhi(ot, o * M, o * M).B(s.Lld.p, 1, M)
        .C(s.Z.p, M, 1, 0, 0.5, 1.0).tag("cc_D2").run(x, p, o64);
  }
  G(Mt, Mt, M).A(s.Z.p, M, 1).Mhi(ot, o * M, o * M).B(uA, 1, M).Nhi(ot, o * M, o)
      .C(R, M, 1, 0, 0.5, 1.0).tag("cc_D2").run(x, p, true);
  // --- E2: Wvv = F_bc - sum uB_bkdl g_ldkc, Woo = F_kj + sum uB_cldj g_kdlc
  s.Wvv.ensure(al, v * v * sizeof(T));
  s.Woo.ensure(al, o * o * sizeof(T));
  {
    const int64_t nv[4] = {1, 1, v, v}, sv[4] = {0, 0, v, 1};
    const int64_t no[4] = {1, 1, o, o}, so[4] = {0, 0, o, 1};
    k::permute4<T, T>(x, off<T>(s.Wvv), static_cast<const T *>(blk[CB_FVV]), nv, sv,
                      incB ? 1.0 : 0.0, 0.0);
    k::permute4<T, T>(x, off<T>(s.Woo), static_cast<const T *>(blk[CB_FOO]), no, so,
                      incB ? 1.0 : 0.0, 0.0);
  }
  if (incQ) {
    s.g2.ensure(al, M * M * sizeof(T));
    s.g3.ensure(al, M * M * sizeof(T));
    const int64_t nn2[4] = {v, o, v, o}, s2[4] = {1, v, M, v * M};   // g2[c][k][d][l]
    const int64_t nn3[4] = {v, o, v, o}, s3[4] = {1, v, M, v * M};   // g3[c][l][d][k]
    k::permute4<T, T>(x, off<T>(s.g2), static_cast<const T *>(blk[CB_OVOV]), nn2, s2, 1.0, 0.0);
    k::permute4<T, T>(x, off<T>(s.g3), static_cast<const T *>(blk[CB_OVOV]), nn3, s3, 1.0, 0.0);
    // Wvv rows b and Woo columns j of the CCSD space (prefixes)
    G(vt, v, o * M).A(uB, o * M, 1).B(s.g2.p, 1, o * M).C(s.Wvv.p, v, 1, 0, -1.0, 1.0)
        .tag("cc_E2").run(x, p, o64);
    G(o, ot, v * o * v).A(s.g3.p, 1, o).B(uB, o, 1).C(s.Woo.p, o, 1, 0, 1.0, 1.0)
        .tag("cc_E2").run(x, p, o64);
  }
  if (full) {
    // rows (a,i,j) of tL: R[(a,i)][(b,j)] += sum_c tA_aicj Wvv[b][c]
    G(M * o, v, v).A(s.tL.p, v, 1).Mhi(o, o * v, M).B(s.Wvv.p, 1, v).C(R, 1, o, 0, 1.0, 1.0)
        .tag("cc_E2").run(x, p, true);
    G(M * v, o, o).A(tA, o, 1).B(s.Woo.p, o, 1).C(R, o, 1, 0, -1.0, 1.0).tag("cc_E2")
        .run(x, p, true);
  } else {
    // the same over the CCSD space, batched over a: rows (i, j) x columns b,
    // then rows (i, b) x columns j
    G(ot * ot, vt, v, 1, vt).A(s.tL.p, v, 1, 0, o * o * v).Mhi(ot, o * v, M)
        .B(s.Wvv.p, 1, v).C(R, 1, o, o * M, 1.0, 1.0).tag("cc_E2").run(x, p, true);
    G(ot * vt, ot, o, 1, vt).A(tA, o, 1, 0, o * M).Mhi(vt, M, M).B(s.Woo.p, o, 1)
        .C(R, o, 1, o * M, -1.0, 1.0).tag("cc_E2").run(x, p, true);
  }
}

template <typename T> void mlcc_problem::ccsd_omega2_t() {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t M = d.M;
  ccsd_integrals_t<T>();
  CcsdState &s = *cc;
  s.tT.ensure(al, M * M * sizeof(T));
  k::convert<T, double>(x, off<T>(s.tT), x2(), M * M);
  double *om2 = om.as<double>() + d.n1;
  s.Rb.ensure(al, M * M * sizeof(double));
  k::fill(x, om2, M * M, 0.0);
  k::fill(x, s.Rb.as<double>(), M * M, 0.0);
  const void *blk[CB_N] = {s.g_vovo.p, s.g_oooo.p, s.g_ovov.p, s.g_oovv.p,
                           s.g_voov.p, s.g_vvvv.p, s.Fvv.p,    s.Foo.p};
  ccsd_terms_t<T>(blk, s.tT.p, u.p, s.tT.p, u.p, true, true, true, true, om2, s.Rb.as<double>());
  k::sym_accum(x, M, s.Rb.as<double>(), om2);
  // three-level: CC2-level projections outside the CCSD space, g~ + eps x
  if (d.cc2_rows())
    k::cc2_rows<T>(x, M, d.o, d.ot, d.vt, off<T>(s.g_vovo), M, false, eps_ai.as<double>(), x2(),
                   M, om2);
}

// Jacobian intermediate for the ladder-integral derivative:
//   Y3[K][i][b][j] = sum_cd g~_Kcbd t_cidj,  g~_Kcbd = sum_J L~^J_Kc L~^J_bd
template <typename T> void mlcc_problem::ccsd_prepare_t() {
  Exec &x = *ex;
  Alloc *al = ex->al;
  CcsdState &s = *cc;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O, o = d.o, v = d.v, M = d.M;
  const int64_t ot = d.ot, vt = d.vt;
  const Prec p = gemm_prec<T>();
  const bool o64 = sizeof(T) == 8;
  if (ot * vt == 0) return;  // no CCSD-level projection
  s.LKc.ensure(al, J * O * v * sizeof(T));
  k::pack2d<T, T>(x, off<T>(s.LKc), off<T>(Lt, O), J, n2, O, v, n);
  // Gk[(K,c)][(b,d)] for b in the CCSD space (leading dimension vt*v)
  s.Gk.ensure(al, (size_t)O * v * vt * v * sizeof(T));
  G(O * v, vt * v, J).A(s.LKc.p, 1, O * v).B(s.Lvv.p, v * v, 1).C(s.Gk.p, vt * v, 1)
      .tag("cc_Gk").run(x, p, o64);
  s.Y3.ensure(al, (size_t)O * o * M * sizeof(T));
  {
    const int64_t nn[4] = {v, o, o, v}, sl[4] = {o * M, M, 1, o};
    s.tL.ensure(al, M * M * sizeof(T));
    k::permute4<T, T>(x, off<T>(s.tL), off<T>(s.tT), nn, sl, 1.0, 0.0);
  }
  // Y3[K][i][b][j] for i, j < ot and b < vt
  G(O * vt, ot * ot, v, v).A(s.Gk.p, v, 1, vt * v).Mhi(vt, v * vt * v, o * M)
      .B(s.tL.p, 1, v, o * o * v).Nhi(ot, o * v, M).C(s.Y3.p, o, 1).tag("cc_Y3").run(x, p, o64);
  s.Gk.release();
}

template <typename T>
void mlcc_problem::ccsd_sigma2_t(const double *c1, const double *c2, const double *Gv,
                                 int64_t ldg, const void *dLvo, int64_t ldl, double *s2) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  CcsdState &s = *cc;
  const int64_t J = d.J, n = d.n, n2 = d.n2, O = d.O, V = d.V, o = d.o, v = d.v, M = d.M;
  const int64_t n1 = d.n1;
  const Prec p = gemm_prec<T>();
  const bool o64 = sizeof(T) == 8;
  const T *lt = off<T>(Lt);
  const double *F = Ft.as<double>();
  s.c1T.ensure(al, n1 * sizeof(T));
  s.c2T.ensure(al, M * M * sizeof(T));
  s.cu2.ensure(al, M * M * sizeof(T));
  T *c1t = off<T>(s.c1T);
  k::convert<T, double>(x, c1t, c1, n1);
  s.c1tt.ensure(al, n1 * sizeof(T));  // c1tt[I][B] = c_BI
  T *c1tt = off<T>(s.c1tt);
  k::pack2d_t<T, double>(x, c1tt, c1, 1, 0, V, O, O);
  k::convert<T, double>(x, off<T>(s.c2T), c2, M * M);
  k::u_of<T>(x, d.o, d.v, c2, off<T>(s.cu2));

  // derivatives of the active L~ blocks: dL_kj = sum_B L~_kB c_Bj,
  // dL_ab = -sum_K c_aK L~_Kb (dL_ai is given, dL_kc = 0)
  s.dLoo.ensure(al, J * o * o * sizeof(T));
  s.dLvv.ensure(al, J * v * v * sizeof(T));
  G(o, o, V, 1, J).A(lt + O, n, 1, 0, n2).B(c1t, O, 1, 0, 0).C(s.dLoo.p, o, 1, o * o)
      .tag("cc_dL").run(x, p, o64);
  G(v, v, O, 1, J).A(c1t, O, 1, 0, 0).B(lt + O, n, 1, 0, n2).C(s.dLvv.p, v, 1, v * v, -1.0)
      .tag("cc_dL").run(x, p, o64);
  // derivative integral blocks
  s.dg_oooo.ensure(al, o * o * o * o * sizeof(T));
  s.dg_oovv.ensure(al, o * o * v * v * sizeof(T));
  s.dg_voov.ensure(al, M * M * sizeof(T));
  G(o * o, o * o, J).A(s.dLoo.p, 1, o * o).B(s.Loo.p, o * o, 1).C(s.dg_oooo.p, o * o, 1)
      .tag("cc_dg").run(x, p, o64);
  G(o * o, o * o, J).A(s.Loo.p, 1, o * o).B(s.dLoo.p, o * o, 1)
      .C(s.dg_oooo.p, o * o, 1, 0, 1.0, 1.0).tag("cc_dg").run(x, p, o64);
  G(o * o, v * v, J).A(s.dLoo.p, 1, o * o).B(s.Lvv.p, v * v, 1).C(s.dg_oovv.p, v * v, 1)
      .tag("cc_dg").run(x, p, o64);
  G(o * o, v * v, J).A(s.Loo.p, 1, o * o).B(s.dLvv.p, v * v, 1)
      .C(s.dg_oovv.p, v * v, 1, 0, 1.0, 1.0).tag("cc_dg").run(x, p, o64);
  G(M, M, J).A(dLvo, 1, ldl).B(s.Lkc.p, M, 1).C(s.dg_voov.p, M, 1).tag("cc_dg").run(x, p, o64);
  // derivative Fock blocks:
  //   dF = F~C - CF~ + 2 sum_K L~^K dX^K - sum_K sum_I (L~^K C)_pI L~^K_Iq,
  //   dX^K = sum_IB L~^K_IB c_BI
  s.dF64.ensure(al, (v * v + o * o) * sizeof(double));
  double *dFvv64 = s.dF64.as<double>(), *dFoo64 = dFvv64 + v * v;
  G(v, v, O).A(c1, O, 1).B(F + O, n, 1).C(dFvv64, v, 1, 0, -1.0).run(x, Prec::F64, true);
  G(o, o, V).A(F + O, n, 1).B(c1, O, 1).C(dFoo64, o, 1).run(x, Prec::F64, true);
  s.dXk.ensure(al, J * sizeof(T));
  G(J, 1, V, O).A(lt + O, n2, 1, n).B(c1t, O, 0, 1).C(s.dXk.p, 1, 0).tag("cc_dF").run(x, p, o64);
  G(1, v, J, 1, v).A(s.dXk.p, 0, 1, 0, 0).B(lt + O * n + O, n2, 1, 0, n)
      .C(dFvv64, 0, 1, v, 2.0, 1.0).tag("cc_dF").run(x, p, true);
  G(1, o, J, 1, o).A(s.dXk.p, 0, 1, 0, 0).B(lt, n2, 1, 0, n).C(dFoo64, 0, 1, o, 2.0, 1.0)
      .tag("cc_dF").run(x, p, true);
  s.Pv.ensure(al, J * v * O * sizeof(T));
  s.Po.ensure(al, J * o * O * sizeof(T));
  G(v, O, V, 1, J).A(lt + O * n + O, n, 1, 0, n2).B(c1tt, 1, V, 0, 0).C(s.Pv.p, O, 1, v * O)
      .tag("cc_dF").run(x, p, o64);
  // L~_Ib = L_Ib = L_bI (the ov block does not depend on t1), read with I contiguous
  G(v, v, O, J).A(s.Pv.p, O, 1, v * O).B(off<T>(L, O * n), 1, n, n2)
      .C(dFvv64, v, 1, 0, -1.0, 1.0).tag("cc_dF").run(x, p, true);
  G(o, O, V, 1, J).A(lt + O, n, 1, 0, n2).B(c1tt, 1, V, 0, 0).C(s.Po.p, O, 1, o * O)
      .tag("cc_dF").run(x, p, o64);
  G(o, o, O, J).A(s.Po.p, O, 1, o * O).B(lt, n, 1, n2).C(dFoo64, o, 1, 0, -1.0, 1.0)
      .tag("cc_dF").run(x, p, true);
  s.dFvv.ensure(al, v * v * sizeof(T));
  s.dFoo.ensure(al, o * o * sizeof(T));
  k::convert<T, double>(x, off<T>(s.dFvv), dFvv64, v * v);
  k::convert<T, double>(x, off<T>(s.dFoo), dFoo64, o * o);

  // sigma_2 = sym + R + R^T, sym starting from dg_vovo = Gv + Gv^T
  s.Rs.ensure(al, M * M * sizeof(double));
  double *Rp = s.Rs.as<double>();
  k::sym_plus_diag<double>(x, M, Gv, ldg, eps_ai.as<double>(), nullptr, s2);
  k::fill(x, Rp, M * M, 0.0);
  // ladder-integral derivative: R += -sum_K c_aK Y3[K][i][b][j]
  if (!d.cc2_rows())
    G(v, o * M, O).A(c1t, O, 1).B(s.Y3.p, o * M, 1).C(Rp, o * M, 1, 0, -1.0, 1.0)
        .tag("cc_Y3c").run(x, p, true);
  else  // over the CCSD space, batched over i: rows a x columns (b, j)
    G(d.vt, (int64_t)d.vt * d.ot, O, 1, d.ot).A(c1t, O, 1, 0, 0).B(s.Y3.p, o * M, 1, 0, M)
        .Nhi(d.ot, o, o).C(Rp, o * M, 1, M, -1.0, 1.0).tag("cc_Y3c").run(x, p, true);
  const void *dblk[CB_N] = {nullptr, s.dg_oooo.p, nullptr, s.dg_oovv.p,
                            s.dg_voov.p, nullptr, s.dFvv.p, s.dFoo.p};
  const void *blk[CB_N] = {s.g_vovo.p, s.g_oooo.p, s.g_ovov.p, s.g_oovv.p,
                           s.g_voov.p, s.g_vvvv.p, s.Fvv.p,    s.Foo.p};
  // (dg, dF; t, t): terms with one amplitude (two-amplitude terms carry g_ovov)
  ccsd_terms_t<T>(dblk, s.tT.p, u.p, s.tT.p, u.p, false, true, false, false, s2, Rp);
  // (g, F; c2, t): terms with at least one amplitude, the first replaced
  ccsd_terms_t<T>(blk, s.c2T.p, s.cu2.p, s.tT.p, u.p, false, true, true, true, s2, Rp);
  // (g, F; t, c2): terms with two amplitudes, the second replaced
  ccsd_terms_t<T>(blk, s.tT.p, u.p, s.c2T.p, s.cu2.p, false, false, true, false, s2, Rp);
  k::sym_accum(x, M, Rp, s2);
  // three-level: CC2-level rows outside the CCSD space, dg~ + eps c2
  if (d.cc2_rows())
    k::cc2_rows<double>(x, M, d.o, d.ot, d.vt, Gv, ldg, true, eps_ai.as<double>(), c2, M, s2);
}
