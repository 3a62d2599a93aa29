/* Driver of the oracle's decompressor for the sanitizer build of the tests.
 * Input file: records of u64 container length, u64 output capacity, then
 * the container bytes.  Each container is copied into a heap buffer of its
 * exact length and decompressed into one of exactly the given capacity, so
 * a read or write outside either is reported.  Output: one return code per
 * record. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/szref.h"

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  for (;;) {
    uint64_t len = 0, cap = 0;
    if (fread(&len, 8, 1, f) != 1) break;
    if (fread(&cap, 8, 1, f) != 1) return 3;
    uint8_t* buf = (uint8_t*)malloc(len ? len : 1);
    void* out = malloc(cap ? cap : 1);
    if (!buf || !out) return 4;
    if (len && fread(buf, 1, len, f) != len) return 3;
    printf("%d\n", szref_decompress(buf, (size_t)len, out, (size_t)cap));
    fflush(stdout); /* a sanitizer abort then shows which record it was */
    free(buf);
    free(out);
  }
  fclose(f);
  return 0;
}
