// nd_peel_gen_b.hip -- peel kernels of the pairs with s = 5..7 and more than
// 9 other r-cliques per s-clique: (2,6) (4,6), (3,6), (2,7) (5,7),
// (3,7) (4,7).
#include "nd_peel_kern.h"

nd_status nd_peel_general_b(nd_ctx *c, PeelArgs &pa, bool te, uint32_t others) {
  switch (others) {
    case 14: return te ? run_te<0, 14>(c, pa) : launch_peel<0, 14, true>(c, pa);
    case 19: return te ? run_te<0, 19>(c, pa) : launch_peel<0, 19, true>(c, pa);
    case 20: return te ? run_te<0, 20>(c, pa) : launch_peel<0, 20, true>(c, pa);
    case 34: return te ? run_te<0, 34>(c, pa) : launch_peel<0, 34, true>(c, pa);
    default: return nd_fail(c, ND_E_UNSUPPORTED, "peeling for this (r,s) is not built");
  }
}
