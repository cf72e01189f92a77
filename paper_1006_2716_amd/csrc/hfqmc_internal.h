// hfqmc_internal.h -- device descriptors shared by the host ABI and the gfx950
// kernels of the Hirsch-Fye QMC engine.  Not part of the public C ABI.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace hfqmc {

// Largest number of time slices: the register-tile kernels handle up to 128,
// the global-memory kernel up to 160.
constexpr int kMaxL = 160;
constexpr int kMaxRegisterL = 128;
// Panel capacity (largest delay depth) of the global-memory kernel.
constexpr int kGlobalMaxDelay = 16;

// Operation a work item performs.
enum Op : int32_t {
  OP_SWEEPS = 0,     // Markov-chain sweeps [sweep_begin, sweep_end) with measurement
  OP_FORCE = 1,      // forced flips of a slice list (deterministic test hook)
  OP_RECOMPUTE = 2,  // from-scratch Dyson recompute only
};

// Item flags.
enum Flags : int32_t {
  F_FIELDS_GIVEN = 1,  // take the initial fields from the init array, else draw them
  F_RESUME = 2,        // load fields and G tiles from the state area (no fresh Dyson)
  F_SAVE = 4,          // store the fields (and with F_SAVE_G the G tiles) at the end
  F_ZERO_ACC = 8,      // clear bins and status before running
  F_KEEP_FIELDS = 16,  // take the fields left in the fields array, fresh Dyson
  F_SAVE_G = 32,       // with F_SAVE: also store the register kernels' G tiles (resumable
                       // sites); a batch solve stores only the fields
};

// One impurity work item.  All offsets are in bytes from the workspace base.
struct alignas(16) ImpDesc {
  int32_t L;                // time slices (<= kMaxL)
  int32_t LT;               // L padded to the kernel's tile multiple
  int32_t op;               // Op
  int32_t flags;            // Flags
  int32_t n_bins;
  int32_t recompute_every;  // sweeps between from-scratch Dyson recomputes
  int32_t n_force;          // OP_FORCE: number of slices
  int32_t delay;            // rank of delayed updates (1 = plain Sherman-Morrison)
  double lam;               // cosh(lam) = exp(dtau U / 2)
  double dflip_p;           // exp(-2 lam) - 1 : flip factor when sigma*s_l = +1
  double dflip_m;           // exp(+2 lam) - 1 : flip factor when sigma*s_l = -1
  double dset_p;            // exp(+lam) - 1   : V from 0 to +lam (Dyson by updates)
  double dset_m;            // exp(-lam) - 1   : V from 0 to -lam
  int64_t n_warmup;
  int64_t n_measure;
  int64_t sweep_begin;      // first sweep this launch runs (global sweep index)
  int64_t sweep_end;        // one past the last
  int64_t rng_offset;       // added to the sweep index in the Philox counter
  uint64_t seed;            // Philox key word 0
  uint64_t site;            // Philox key word 1
  int64_t off_weiss;        // 2 x L doubles: g_up(tau_k), g_dn(tau_k)
  int64_t off_fields;       // L int8 fields (in and out)
  int64_t off_bins;         // n_bins x NV doubles: per-bin sums (accumulated)
  int64_t off_status;       // ImpStatus
  int64_t off_state;        // 4 x LT x LT + 256 doubles: G of both spins (register kernels:
                            // tiles in lane order; global kernel: row-major), then the drift
                            // snapshot (global kernel) or parked bin sums (register kernels)
  int64_t off_force;        // OP_FORCE: n_force int32 slices, then n_force doubles ratios
  int64_t off_init;         // F_FIELDS_GIVEN: L int8 initial fields (read only)
  int64_t chain;            // chain index of this impurity: Philox counter word 3
  double drift_limit;       // > 0: a scheduled recompute that measures more drift halves
                            // the interval to the next one; at interval 1 it is an error
  int64_t poison[2];        // test hook, 0 = none: the ratios of the first attempt of sweep
                            // poison[0] - 1 and of the repeated attempt of sweep
                            // poison[1] - 1 read a NaN-poisoned diagonal of G
};

struct alignas(16) ImpStatus {
  int64_t proposals;
  int64_t accepts;
  int64_t nonpositive;
  int64_t error;            // nonzero: non-finite ratio or Green function seen and not
                            // recovered, or the drift limit exceeded at one sweep
  double max_drift;         // max |G_updated - G_recomputed| over recomputes
  int64_t next_rec;         // drift limit on: sweep of the next from-scratch Dyson solve
  int32_t rec_every;        // drift limit on: current sweeps between Dyson solves (0: unset)
  int32_t recoveries;       // sweeps repeated after a ratio that was not a positive number,
                            // each from a from-scratch Dyson solve of its starting fields
  double pad;
};

// Number of measured values per bin: g_up(0..L), g_dn(0..L), n_up, n_dn, d.
__host__ __device__ inline int n_values(int L) { return 2 * (L + 1) + 3; }

}  // namespace hfqmc
