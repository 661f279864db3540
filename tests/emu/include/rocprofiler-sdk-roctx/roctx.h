// Host emulation build: ROCTX ranges are no-ops.  Test infrastructure only.
#pragma once
inline int roctxRangePushA(const char *) { return 0; }
inline int roctxRangePop() { return 0; }
