// zt_epi_plain.hip -- the z,t synthesis kernel variants of the ZEPI_PLAIN epilogue (zt_epi.h).
#include "zt_epi.h"

namespace fno {
FNO_ZT_INSTANTIATE(ZEPI_PLAIN)
}  // namespace fno
