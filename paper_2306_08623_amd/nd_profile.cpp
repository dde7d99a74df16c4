// nd_profile -- runs the decomposition through the C ABI from a plain C++
// program (no Python, no PyTorch), for profilers that must own the process.
//
//   nd_profile <graph.csr> <r> <s> [steps] [work_chunk] [peel_blocks] [el|te]
//
// The graph file is the binary CSR written by inputs.save_csr():
// uint32 n, uint64 nnz, uint64 row_ptr[n+1], uint32 col[nnz] (little endian).
// Prints one line of statistics per decomposition.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "nucleus.h"

int main(int argc, char **argv) {
  if (argc < 4) {
    std::fprintf(stderr, "usage: %s graph.csr r s [steps]\n", argv[0]);
    return 2;
  }
  const uint32_t r = (uint32_t)std::atoi(argv[2]), s = (uint32_t)std::atoi(argv[3]);
  const int steps = argc > 4 ? std::atoi(argv[4]) : 1;
  const uint32_t chunk = argc > 5 ? (uint32_t)std::atoi(argv[5]) : 0;
  const uint32_t blocks = argc > 6 ? (uint32_t)std::atoi(argv[6]) : 0;
  const std::string mode = argc > 7 ? argv[7] : "";
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) {
    std::perror("open");
    return 1;
  }
  uint32_t n = 0;
  uint64_t nnz = 0;
  if (std::fread(&n, 4, 1, f) != 1 || std::fread(&nnz, 8, 1, f) != 1) return 1;
  std::vector<uint64_t> rp(n + 1ull);
  std::vector<uint32_t> col(nnz ? nnz : 1);
  if (std::fread(rp.data(), 8, n + 1ull, f) != n + 1ull) return 1;
  if (nnz && std::fread(col.data(), 4, nnz, f) != nnz) return 1;
  std::fclose(f);
  nd_ctx *ctx = nullptr;
  nd_options opt = {};
  opt.validate = 1;
  opt.work_chunk = chunk;
  opt.peel_blocks = blocks;
  if (mode == "el") opt.flags |= ND_FLAG_HIER_EL;
  if (mode == "te") opt.flags |= ND_FLAG_HIER_TE;
  nd_status st = nd_create(&ctx, &opt);
  if (st != ND_OK) {
    std::fprintf(stderr, "nd_create: %s (%s)\n", nd_status_str(st), nd_last_error(nullptr));
    return 1;
  }
  st = nd_load_csr(ctx, n, nnz, rp.data(), col.data(), ND_MEM_HOST);
  if (st == ND_OK) st = nd_set_rs(ctx, r, s);
  for (int i = 0; st == ND_OK && i < steps; i++) {
    st = nd_decompose(ctx);
    nd_info info;
    if (st == ND_OK && (st = nd_get_info(ctx, &info)) == ND_OK)
      std::printf("step %d: n_r=%llu n_s=%llu k=%u rounds=%u prep=%.3f count=%.3f peel=%.3f "
                  "tree=%.3f ms (count kernel %.3f, peel kernel %.3f, hierarchy %.3f) "
                  "link_calls=%llu link_steps=%llu cas_retries=%llu grid_retries=%u "
                  "n_int=%llu\n",
                  i, (unsigned long long)info.n_r, (unsigned long long)info.n_s, info.k,
                  info.rounds, info.ms_prep, info.ms_count, info.ms_peel, info.ms_tree,
                  info.ms_count_kernel, info.ms_peel_kernel, info.ms_hier,
                  (unsigned long long)info.link_calls, (unsigned long long)info.links,
                  (unsigned long long)info.cas_retries, info.grid_retries,
                  (unsigned long long)info.n_int);
    std::fflush(stdout);
  }
  if (st != ND_OK) std::fprintf(stderr, "error: %s (%s)\n", nd_status_str(st), nd_last_error(ctx));
  nd_destroy(ctx);
  return st == ND_OK ? 0 : 1;
}
