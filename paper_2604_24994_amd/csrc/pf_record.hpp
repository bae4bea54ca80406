// Field packing of the contribution records (plain integer code: the kernels
// compile it for the device, the host tests compile it with a host compiler).
//
// The fourth word of a record holds the view (12 bits, 0..4095) and the two
// binding constraints of the contribution's interval (10 bits each, stored
// as b + 2 so that -2 = ray start and -1 = sphere fit; f >= 0 is a raster
// face index, f <= 1021).  The word is packed and unpacked as an unsigned
// value, so views 2048..4095 (bit 31 set) decode as themselves.
#pragma once

#include <cstdint>

#ifndef PF_HD
#define PF_HD
#endif

namespace pf {

constexpr int REC_MAX_VIEWS = 4096;   // views per call that a forward state can record
constexpr int REC_MAX_BIND = 1021;    // largest face index a record can name

PF_HD inline int32_t pack_view_bind(int view, int bind0, int bind1) {
  return (int32_t)(((uint32_t)view << 20) | ((uint32_t)(bind0 + 2) << 10) | (uint32_t)(bind1 + 2));
}
PF_HD inline int rec_view(int32_t w) { return (int)((uint32_t)w >> 20); }
PF_HD inline int rec_bind0(int32_t w) { return (int)(((uint32_t)w >> 10) & 1023u) - 2; }
PF_HD inline int rec_bind1(int32_t w) { return (int)((uint32_t)w & 1023u) - 2; }

}  // namespace pf
