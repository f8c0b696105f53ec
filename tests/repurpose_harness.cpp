// Test harness (host only): runs the library's host walk of subpixel repurposing (Alg. 2) on a view map read
// from a file and writes the source pixel of every subpixel.
//   usage: repurpose_harness W H N a b p q r c pw V.u8 out.i32
// with tan(alpha) = a/b, L_x = p/q, K_offset = r/c; V.u8 holds V[H][3W] (uint8); out.i32 receives src[H][W][3]
// (x' W + y').  Exit status: 0, or the library's error code (message on stderr).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_2407_14053_amd/csrc/dl_internal.h"

int main(int argc, char** argv) {
  if (argc != 13) return 2;
  dl_display_desc d{};
  d.width = std::atoi(argv[1]);
  d.height = std::atoi(argv[2]);
  d.n_views = std::atoi(argv[3]);
  d.tan_slant = {std::atoll(argv[4]), std::atoll(argv[5])};
  d.pitch = {std::atoll(argv[6]), std::atoll(argv[7])};
  d.offset = {std::atoll(argv[8]), std::atoll(argv[9])};
  const int pw = std::atoi(argv[10]);
  const size_t n = (size_t)d.height * 3 * d.width;
  std::vector<uint8_t> V(n);
  FILE* f = std::fopen(argv[11], "rb");
  if (!f || std::fread(V.data(), 1, n, f) != n) return 3;
  std::fclose(f);
  std::vector<int32_t> src(n);
  std::string why;
  const int rc = dl::repurpose_sources(d, pw, V.data(), src.data(), &why);
  if (rc) {
    std::fprintf(stderr, "%s\n", why.c_str());
    return 10 - rc;
  }
  FILE* g = std::fopen(argv[12], "wb");
  if (!g || std::fwrite(src.data(), 4, n, g) != n) return 4;
  std::fclose(g);
  return 0;
}
