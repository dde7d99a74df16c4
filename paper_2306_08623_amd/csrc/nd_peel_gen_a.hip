// nd_peel_gen_a.hip -- peel kernels of the pairs with s = 5..7 and at most
// 9 other r-cliques per s-clique: (1,5) (4,5), (1,6) (5,6), (1,7) (6,7),
// (2,5) (3,5). (Split from nd_peel_gen_b.hip so the two compile in
// parallel.)
#include "nd_peel_kern.h"

nd_status nd_peel_general_a(nd_ctx *c, PeelArgs &pa, bool te, uint32_t others) {
  switch (others) {
    case 4: return te ? run_te<0, 4>(c, pa) : launch_peel<0, 4, true>(c, pa);
    case 5: return te ? run_te<0, 5>(c, pa) : launch_peel<0, 5, true>(c, pa);
    case 6: return te ? run_te<0, 6>(c, pa) : launch_peel<0, 6, true>(c, pa);
    case 9: return te ? run_te<0, 9>(c, pa) : launch_peel<0, 9, true>(c, pa);
    default: return nd_fail(c, ND_E_UNSUPPORTED, "peeling for this (r,s) is not built");
  }
}
