// Instantiations of the tuned exact kernel (exact_v2_body.h) for one variant
// and a range of n.  The build compiles this file several times with
//   -DSK_V2_VARIANT=v -DSK_V2_NMIN=a -DSK_V2_NMAX=b
// so the specialisations compile in parallel; each registers itself with the
// host-side kernel table at load time.
#include "exact_v2_body.h"

namespace sk {

using ExactV2Fn = void (*)(const ExactArgsV2, double*);
int register_exact_v2(int variant, int n, int nprimes, int inner, ExactV2Fn fn);

// Inner (fully unrolled) walk variables per instance.  Four in general; three
// for Skolem n = 22..25, whose scalar pair-sum state (B and the N_q of the
// inner variables) overflows the SGPR file at four: the compiled 16-step
// block issues 2-3 % fewer VALU instructions per sign vector than the 32-step
// one there (S(24): 57.5 against 58.8), while for the Langford instances of
// the same size and for n >= 26 the longer block is the better one.
template <int V, int N>
constexpr int inner_for()
{
    return (V == 0 && N >= 22 && N <= 25) ? 3 : 4;
}

template <int V, int N>
constexpr bool v2_supported()
{
    constexpr PlanCE P = make_plan_ce(N, V);
    return P.ok && P.n_lane == 6 && P.n_walk >= inner_for<V, N>() + 1;
}

template <int V, int N>
int register_one()
{
    if constexpr (v2_supported<V, N>()) {
        constexpr int I = inner_for<V, N>();
        return register_exact_v2(V, N, primes_for(N), I, exact_v2_kernel<V, N, primes_for(N), I>);
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
