// Instantiations of the tuned exact kernel (exact_v2_body.h) for one variant
// and a range of n.  The build compiles this file several times with
//   -DSK_V2_VARIANT=v -DSK_V2_NMIN=a -DSK_V2_NMAX=b
// so the specialisations compile in parallel; each registers itself with the
// host-side kernel table at load time.
#include "exact_v2_body.h"

namespace sk {

using ExactV2Fn = void (*)(const ExactArgsV2, double*);
int register_exact_v2(int variant, int n, int nprimes, int inner, ExactV2Fn fn);

constexpr int kInner = 4;

template <int V, int N>
constexpr bool v2_supported()
{
    constexpr PlanCE P = make_plan_ce(N, V);
    return P.ok && P.n_lane == 6 && P.n_walk >= kInner + 1;
}

template <int V, int N>
int register_one()
{
    if constexpr (v2_supported<V, N>()) {
        return register_exact_v2(V, N, primes_for(N), kInner, exact_v2_kernel<V, N, primes_for(N), kInner>);
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
