// ppt_half.h -- outward rounding of BVH box bounds to IEEE binary16 (host side).
//
// A box bound stored as a half float is rounded away from the box's inside: half_down(x) <= x <=
// half_up(x), with equality when x is a half float, and the two never more than one half-float
// step apart.  Beyond the half range a bound becomes infinite (the box is then unbounded along
// that axis, still conservative).  Header-only so that a host test can compile it on its own.
#ifndef PPT_HALF_H
#define PPT_HALF_H

#include <cstdint>
#include <cstring>

namespace ppt {

inline uint16_t half_bits(_Float16 h) { uint16_t b; std::memcpy(&b, &h, 2); return b; }
inline float half_value(uint16_t b) { _Float16 h; std::memcpy(&h, &b, 2); return (float)h; }
inline uint16_t half_down(float x) {
    const uint16_t b = half_bits((_Float16)x);  // nearest
    if (half_value(b) <= x) return b;
    if (b == 0x0000u) return 0x8001u;           // +0 above a tiny negative x
    return (b & 0x8000u) ? (uint16_t)(b + 1) : (uint16_t)(b - 1);
}
inline uint16_t half_up(float x) {
    const uint16_t b = half_bits((_Float16)x);
    if (half_value(b) >= x) return b;
    if (b == 0x8000u) return 0x0001u;           // -0 below a tiny positive x
    return (b & 0x8000u) ? (uint16_t)(b - 1) : (uint16_t)(b + 1);
}

}  // namespace ppt

#endif
