// The per-target code of dimension PCMS_EMU_DIM, for the CPU emulation
// (compiled once per dimension).
#include "emu_common.h"

namespace emu {

template <>
void dispatch_dim<PCMS_EMU_DIM>(int op, const KArgs &a, const GridParams &gp, int group,
                                int degree, int precision, bool unit)
{
    if (unit) dispatch<PCMS_EMU_DIM, true>(op, a, gp, group, degree, precision);
    else dispatch<PCMS_EMU_DIM, false>(op, a, gp, group, degree, precision);
}

}  // namespace emu
