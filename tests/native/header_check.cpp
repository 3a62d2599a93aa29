// Host-only driver of the container header checks (parse_header and
// check_sections of the library's container.hpp), built by the tests with a
// host compiler and the address and undefined-behaviour sanitizers.
//
// Input file: records of a u64 claimed container size followed by the
// 192 header bytes.  Output: one line per record with the two return codes.
#include <stdio.h>

#include <vector>

#include "../../paper_1706_03791_amd/csrc/container.hpp"

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  for (;;) {
    uint64_t size = 0;
    if (fread(&size, 8, 1, f) != 1) break;
    // an exact-size heap copy, so any read past the header is caught
    std::vector<uint8_t> hdr(szh::kHdr);
    if (fread(hdr.data(), 1, szh::kHdr, f) != szh::kHdr) return 3;
    szh::Hdr h;
    const int a = szh::parse_header(hdr.data(), (size_t)size < szh::kHdr ? (size_t)size : szh::kHdr, h, false);
    int b = a;
    if (!a) {
      b = szh::check_sections(h);
      if (!b && h.total > size) b = SZ_ECORRUPT;
    }
    printf("%d %d\n", a, b);
  }
  fclose(f);
  return 0;
}
