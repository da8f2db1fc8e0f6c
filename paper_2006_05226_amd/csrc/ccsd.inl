// MLCCSD (CCS/CCSD) doubles: residual and Jacobian doubles (included by problem.cpp).
template <typename T> void mlcc_problem::ccsd_omega2_t() {
  throw Error{MLCC_E_ARG, "MLCCSD doubles residual not built yet"};
}
template <typename T> void mlcc_problem::ccsd_prepare_t() {
  throw Error{MLCC_E_ARG, "MLCCSD Jacobian not built yet"};
}
template <typename T> void mlcc_problem::ccsd_sigma2_t(const double *, const double *, double *) {
  throw Error{MLCC_E_ARG, "MLCCSD Jacobian not built yet"};
}
template <typename T> void mlcc_problem::ccsd_sigma1_doubles_t(const double *, double *) {}
