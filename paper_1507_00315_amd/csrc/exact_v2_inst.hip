// Instantiations of the tuned exact kernel (exact_v2_body.h) for one variant
// and a range of n.  The build compiles this file several times with
//   -DSK_V2_VARIANT=v -DSK_V2_NMIN=a -DSK_V2_NMAX=b [-DSK_V2_LARSEN=1]
// so the specialisations compile in parallel; each registers itself with the
// host-side kernel table at load time.  SK_V2_LARSEN=1 builds the
// inclusion-exclusion sum instead of the sign sum.
#include "exact_v2_body.h"

#ifndef SK_V2_LARSEN
#define SK_V2_LARSEN 0
#endif

namespace sk {

using ExactV2Fn = void (*)(const ExactArgsV2);
int register_exact_v2(int variant, int n, int nprimes, int inner, bool larsen, ExactV2Fn fn);

constexpr int kInner = 4;
constexpr bool kLarsen = SK_V2_LARSEN != 0;

template <int V, int N>
constexpr bool v2_supported()
{
    constexpr PlanCE P = make_plan_ce(N, V, kWalkCap, kLarsen);
    return P.ok && P.n_lane == 6 && P.n_walk >= kInner + 1;
}

template <int V, int N>
int register_one()
{
    if constexpr (v2_supported<V, N>()) {
        return register_exact_v2(V, N, primes_for(N), kInner, kLarsen,
                                 exact_v2_kernel<V, N, primes_for(N), kInner, kLarsen>);
    } else {
        return 0;
    }
}

template <int V, int LO, int HI>
int register_range()
{
    if constexpr (LO <= HI) {
        return register_one<V, LO>() + register_range<V, LO + 1, HI>();
    } else {
        return 0;
    }
}

static const int registered = register_range<SK_V2_VARIANT, SK_V2_NMIN, SK_V2_NMAX>();

}  // namespace sk
