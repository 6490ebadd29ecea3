// zt_epi_bwd.hip -- the z,t synthesis kernel variants of the ZEPI_BWD epilogue (zt_epi.h).
#include "zt_epi.h"

namespace fno {
FNO_ZT_INSTANTIATE(ZEPI_BWD)
}  // namespace fno
