// Device side of the best-first frontier (best_first.hip): nodes are records
// (bound, depth, slot) kept sorted by (bound, insertion order) in one of two
// ping-pong arrays; their rows live in a slab and free slots on a stack.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fspbb {

struct Frontier {
    int32_t *lb, *depth, *slot;
};

// sel[0] = number of records with bound < ub (the eliminated ones are the
// tail, the records being sorted by bound), sel[1] = parents taken from the
// front (children fit in pool_cap; the first always), sel[2] = their children.
hipError_t bf_select(const Frontier &F, int64_t M, int32_t ub, int n, int64_t pool_cap, int64_t *sel,
                     hipStream_t s);

// freelist[i] = first + i for i < count.
hipError_t bf_fill_slots(int32_t *freelist, int64_t count, int32_t first, hipStream_t s);

// Orders the survivors of a step by bound, keeping child order on ties: sets
// keys[r] = lb[r] for r < *nsurv and a padding key >= ub beyond (up to cap),
// then sorts (key, rank) pairs stably on the bits of ub into keys_out /
// rank_out (every survivor's bound is below ub).  tmp is grown as needed.
hipError_t bf_sort_survivors(const int32_t *lb, const uint32_t *nsurv, int64_t cap, int32_t ub, int32_t *keys,
                             int32_t *ranks, int32_t *keys_out, int32_t *rank_out, void **tmp, size_t *tmp_bytes,
                             hipStream_t s);

// Merges the remaining records A = F[a0, a0 + nA) with the *nsurv sorted
// survivors (sorted bounds kb, ranks rk; survivor rank r has depth sdep[r] and
// row slot freelist[top - 1 - r]) into G[0, nA + *nsurv); on equal bounds A
// comes first (it was inserted earlier).
hipError_t bf_merge(const Frontier &F, int64_t a0, int64_t nA, const int32_t *kb, const int32_t *rk,
                    const int32_t *sdep, const uint32_t *nsurv, int64_t cap, const int32_t *freelist, int64_t top,
                    const Frontier &G, hipStream_t s);

// Returns the slots of the records F[0, K) (the parents) and F[Mp, M) (the
// eliminated) to the free stack at freelist[top - *nsurv ...].
hipError_t bf_free_slots(const Frontier &F, int64_t K, int64_t Mp, int64_t M, int32_t *freelist, int64_t top,
                         const uint32_t *nsurv, hipStream_t s);

}  // namespace fspbb
