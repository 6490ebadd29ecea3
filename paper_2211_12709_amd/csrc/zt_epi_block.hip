// zt_epi_block.hip -- the z,t synthesis kernel variants of the ZEPI_BLOCK epilogue (zt_epi.h).
#include "zt_epi.h"

namespace fno {
FNO_ZT_INSTANTIATE(ZEPI_BLOCK)
}  // namespace fno
