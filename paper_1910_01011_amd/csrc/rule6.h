// The 6-point degree-4 symmetric triangle rule (Strang-Fix / Dunavant 1985),
// the far rule of every regular pair: barycentric coordinates (two orbits of
// three points) and weights, which sum to 1 (integral = |T| sum_q w_q f(x_q)).
// One definition for every kernel translation unit of the library; each unit
// gets its own copy in constant memory.
#pragma once

#include <hip/hip_runtime.h>

namespace bem {

static __constant__ double q6_bary[6][3] = {
    {0.10810301816807022736, 0.44594849091596488632, 0.44594849091596488632},
    {0.44594849091596488632, 0.10810301816807022736, 0.44594849091596488632},
    {0.44594849091596488632, 0.44594849091596488632, 0.10810301816807022736},
    {0.81684757298045851308, 0.091576213509770743460, 0.091576213509770743460},
    {0.091576213509770743460, 0.81684757298045851308, 0.091576213509770743460},
    {0.091576213509770743460, 0.091576213509770743460, 0.81684757298045851308}};
static __constant__ double q6_w[6] = {0.22338158967801146570, 0.22338158967801146570, 0.22338158967801146570,
                                      0.10995174365532186764, 0.10995174365532186764, 0.10995174365532186764};

}  // namespace bem
