// Learned warm start for the GMRES density (placeholder until the network kernels land).
#include <stdexcept>

#include "solver.h"

using namespace kfbi;

void mlp_release(bidomain_s *b) { b->mlp = nullptr; }
bool mlp_warm_start(bidomain_s *, const double *, const double *, double *, hipStream_t) { return false; }
void mlp_record(bidomain_s *, const double *, const double *, const double *, hipStream_t) {}
void bidomain_s::mlp_init(int, uint64_t) { throw std::invalid_argument("learned warm start not built"); }
double bidomain_s::mlp_train(int, double, hipStream_t) { return 0.0; }
int bidomain_s::mlp_params(float *, int64_t *) { return KFBI_EINVAL; }
