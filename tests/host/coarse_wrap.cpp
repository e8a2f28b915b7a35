// Flat C wrapper of the coarse-level builder for the host-side tests.
#include "coarse.h"
#include <cstring>
extern "C" int coarse_build(int nv, const int* nfree, const double* X, const double* mass, int nt, const int* tv,
                            const double* Dminv, const double* vol, double h, double mu, double lam, int nblk,
                            const int* tn_b0, int max_agg, int* blk_agg, int* nagg, int* agg_b0, int* agg_b1,
                            double* d, double* ainv) {
  tc::CoarseScene cs;
  cs.node0 = 0; cs.nv = nv; cs.nfree = nfree; cs.X = X; cs.mass = mass; cs.tet0 = 0; cs.tet1 = nt; cs.tv = tv;
  cs.Dminv = Dminv; cs.vol = vol; cs.h = h; cs.mu = mu; cs.lam = lam; cs.tn_b0 = tn_b0; cs.bfirst = 0;
  cs.bend = nblk; cs.block = 64; cs.max_agg = max_agg;
  std::vector<int> ba(nblk, -1), b0, b1;
  std::vector<double> dd(3 * (size_t)nv, 0.0), ai;
  const int m = tc::build_coarse(cs, ba, b0, b1, dd, ai);
  std::memcpy(blk_agg, ba.data(), sizeof(int) * nblk);
  *nagg = (int)b0.size();
  std::memcpy(agg_b0, b0.data(), sizeof(int) * b0.size());
  std::memcpy(agg_b1, b1.data(), sizeof(int) * b1.size());
  std::memcpy(d, dd.data(), sizeof(double) * dd.size());
  std::memcpy(ainv, ai.data(), sizeof(double) * ai.size());
  return m;
}
