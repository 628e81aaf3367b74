// The aggregation chain of the AMG setup on the device: the pairwise passes
// and Galerkin products of every level, with the same aggregates and the
// same coarse matrices, bit for bit, as the host chain of msp_host.h.
//
// A pairwise pass visits rows in ascending order and pairs each free
// eligible row with its strongest free eligible candidate (lowest index among
// equals).  Row i only ever pairs with a candidate j > i (every lower row is
// already placed when i is visited), so the pass is the greedy maximal
// matching of the directed edge list {(i, j) : j a candidate of i, j > i}
// taken in the order (i ascending, candidate rank ascending).  That matching
// is the lexicographically first maximal matching for this edge order, and
// it is also what repeated rounds of "take every free edge that comes first
// at both of its endpoints" produce; the device pass runs those rounds.  The
// smallest free row always decides in a round, so there are at most n rounds.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <functional>

#include "msp_host.h"

namespace msp {

// Device memory for the chain's work arrays (freed by the caller after the
// setup; may throw).
using DeviceAlloc = std::function<void *(size_t)>;
// Page-locked host memory of at least `bytes` for the copy of level l (the
// same l never gets a buffer twice in one call); valid until the caller's
// setup ends.  May return nullptr: the copy then goes to pageable memory.
using PinnedBuffer = std::function<void *(int l, size_t bytes)>;
// Called with every HIP error; must not return (it throws).
using HipFail = void (*)(hipError_t);

// Builds the hierarchy of A0 on `st`.  A0 is the host copy of level 0 and
// rp0/ci0/val0 the same matrix in device memory.  Same contract as
// build_hierarchy (with_colors = false): H.A holds every level on the host,
// H.agg every aggregation map, on_smoothed is called for each smoothed level
// as soon as it is known (from another thread for all but the first level:
// the host copy of a level runs on a copy thread, on `copy_st`, while the
// device builds the next one); returns 0 or -9.  The zero-diagonal test of
// build_hierarchy is left to the caller (check_diagonals), so that the
// coarsest-level work can start first.  A0's values may still be on their
// way to the host: level0_values() is called (and must return only once they
// are there) before they are read here, and before returning when level 0 is
// the coarsest level.  Returns 1 without touching
// A0 or H when the level-0 pattern is not structurally symmetric (the pass
// reads a_ji through the mirror entry); the caller then runs the host chain.
// `cap` is an idle stream used only to capture batches of matching rounds
// into a graph (nothing runs on it).  `pinned` is a host-pinned buffer of at
// least 16 ints.  With `staging`, each new level is copied to page-locked
// memory first (a fast DMA), on_smoothed gets its pattern there (so the
// level's host work starts before the copy into H.A is done), and H.A is
// filled from it.  A stalled level (the two passes keep more than 90% of its
// rows) is finished on the host with absorb_singletons and galerkin, and its
// coarse matrix uploaded.
// Bytes of the one device allocation the chain makes for a level 0 of n0
// rows and nnz0 entries (freed with the setup's other temporaries).
size_t device_chain_bytes(int n0, long long nnz0);

int device_hierarchy(Csr &A0, const int *rp0, const int *ci0, const double *val0,
                     int max_coarse, int max_levels, int max_dense, Hierarchy &H,
                     const LevelCallback &on_smoothed, const std::function<void()> &level0_values,
                     hipStream_t st, hipStream_t cap, hipStream_t copy_st,
                     const DeviceAlloc &alloc, HipFail hip_fail, int *pinned,
                     const PinnedBuffer &staging = nullptr);

}  // namespace msp
