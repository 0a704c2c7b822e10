// ms_internal.h -- layout of columns in device memory and the kernel-argument views.
//
// A column lives in one device buffer:
//   [header 256 B][section 0][section 1]...  (every section 256-byte aligned)
//   UNCOMPR:      values[n_cap]
//   STATIC_BP:    rem[32] | payload[n_cap words + slack]
//   DYN_BP family widths[nb_cap] u8 | offsets[nb_cap] | bases[nb_cap] | rem[512] |
//                 payload[nb_cap * 512 words + slack]   (block k may use its 512-word
//                 slot k, or any offset recorded in the block directory)
//   RLE:          rvalues[n_cap] | rstarts[n_cap]
// The header holds every size that a kernel learns only on the device.
#pragma once
#include <stdint.h>

namespace ms {

constexpr int kBlk = 512;           // DynBP-family block size; every kernel walks 512-value chunks
constexpr int kSbpGroup = 32;       // static BP block size
constexpr int kWG = 256;            // threads per workgroup
constexpr int kWaves = kWG / 64;
constexpr uint64_t kPayloadSlackWords = 1024;  // lane windows may read past a section's last word

struct ColHdr {
  unsigned long long n;        // element count
  unsigned long long runs;     // RLE runs
  unsigned int sbp_width;      // static BP width
  unsigned int or_all;         // OR of all values
  unsigned int or_main;        // OR of the compressed main part
  unsigned int sorted;         // 1 when strictly increasing
  unsigned int pad[56];
};
static_assert(sizeof(ColHdr) == 256, "header is 256 bytes");

// Kernel argument view of a column (pointers into its buffer).
struct ColView {
  unsigned int kind;
  unsigned int width;          // static BP: width requested for an output (host-known); inputs read hdr
  ColHdr *hdr;
  unsigned char *widths;
  unsigned int *offsets;
  unsigned int *bases;
  unsigned int *payload;
  unsigned int *rem;
  unsigned int *rvalues;
  unsigned int *rstarts;
  unsigned long long n_cap;    // capacity in values
  unsigned long long payload_cap;  // payload words the buffer holds (readers may touch kPayloadSlackWords more)
};

enum Kind : unsigned { UNCOMPR = 0, STATIC_BP = 1, DYN_BP = 2, DELTA_DYN_BP = 3, FOR_DYN_BP = 4, RLE = 5 };
enum Err : unsigned { E_OK = 0, E_INVALID = 1, E_UNSUPPORTED = 2, E_TOO_WIDE = 3, E_RANGE = 4, E_NOT_SORTED = 5,
                      E_LENGTH = 6 };

inline bool is_dynbp(unsigned k) { return k == DYN_BP || k == DELTA_DYN_BP || k == FOR_DYN_BP; }

}  // namespace ms
