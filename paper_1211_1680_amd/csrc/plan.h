// Host-side table builders (plan.cpp).
#pragma once
#include <vector>

#include "common.h"

namespace s2let {
hipError_t build_sht_tables(int k, ShtTables* T);
void free_sht_tables(ShtTables* T);
hipError_t build_leg_tables(int Lt, LegTables* G);
void free_leg_tables(LegTables* G);
void leg_factors_host(int Lt, std::vector<double>* alpha, std::vector<double>* beta,
                      std::vector<double>* dfac, std::vector<double>* cm);
double k_lambda_host(double t, double lam);
void tiling_host(int L, int B, int J_min, int J, double* kappa, double* eta);
void tiling_host_kernel(int L, int B, int J_min, int J, int kernel, double* kappa, double* eta);
}  // namespace s2let
