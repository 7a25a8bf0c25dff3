// tables.h -- host tabulation of the material models (see tables.cpp).
#pragma once

#include <string>
#include <vector>

#include "mcx.h"

namespace mcx {

struct BuiltTables {
  int n = 0;
  double lemin = 0, dl = 0;
  std::vector<double> block;  // T_NCH * n channel-major, then kSoftN soft-law guesses
  double thr_pp = 0, thr_in[2] = {0, 0}, thr_br = 0;
  double k_coef = 0, eta_a = 0, eta_b = 0, ray_a = 0;
  // soft energy-loss straggling (see Tab in mcx_internal.h)
  double strag_k = 0, strag_b = 0, wcc_soft = 0, wcr_soft = 0;
  double annih_k = 0;  // pi r_e^2 n_e: Heitler's cross section per gram is annih_k times a function of E
};

bool build_tables(const mcx_material_desc& m, const mcx_transport& t, BuiltTables* out, std::string* err);

}  // namespace mcx
