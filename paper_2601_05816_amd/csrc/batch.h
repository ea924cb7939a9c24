// Persistent multi-lattice Wilson kernel (batch.hip).
#pragma once

#include "common.h"
#include "site.h"

namespace lq {

// One problem of a batch: full operator (parity < 0: out = alpha in + beta
// hop(in)) or one odd-even half (out on parity `parity` = alpha xin + beta
// hop(in), in on the other parity).  Blocks are rhs-innermost.
struct batch_prob {
  geo4 g;
  const void* U;
  const void* in;
  const void* xin;
  void* out;
  const int* live;
  int nrhs;
  int parity;
  double alpha, beta;
  unsigned long long unit0;  // first work unit (filled by wilson_batch)
};

struct batch_desc {
  int n;
  unsigned long long total_units;
  batch_prob p[LQCD_MAX_BATCH];
};

geo4 make_geo4(const lqcd_lattice* lat);
hipError_t wilson_batch(batch_desc& d, int prec, bool dagger, hipStream_t s);
void set_batch_grid(int blocks);

}  // namespace lq
