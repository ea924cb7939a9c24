// Persistent multi-lattice Wilson kernel (batch.hip).
#pragma once

#include "common.h"
#include "pencil.h"
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
  pencil_geo pg;             // pencil decomposition (pencil batch kernel; filled by wilson_batch)
  int nr;                    // rhs per work item of the pencil body (1 or 2)
  int ncw;                   // > 0: links of a step through LDS (variant 2), NCW of that body
};

struct batch_desc {
  int n;
  int pl;  // some unit stages its links in LDS (filled by wilson_batch)
  unsigned long long total_units;
  batch_prob p[LQCD_MAX_BATCH];
};

geo4 make_geo4(const lqcd_lattice* lat);
hipError_t wilson_batch(batch_desc& d, int prec, bool dagger, hipStream_t s);
void set_batch_grid(int blocks);
// Residency cap of the pencil batch launch (workgroups per CU, 0 = none).
void set_batch_occupancy(int occ);
// Kernel of the batch launch: 0 automatic (pencils for full-lattice
// applies, one (site, rhs) per work item for odd-even passes), 1 one
// (site, rhs) per work item, 2 time-streaming pencils.
void set_batch_kernel(int kind);
int batch_kernel();

}  // namespace lq
