// zt_epi_adj.hip -- the z,t synthesis kernel variants of the ZEPI_ADJ, ZEPI_ADJ_ACC epilogues (zt_epi.h).
#include "zt_epi.h"

namespace fno {
FNO_ZT_INSTANTIATE(ZEPI_ADJ)
FNO_ZT_INSTANTIATE(ZEPI_ADJ_ACC)
}  // namespace fno
