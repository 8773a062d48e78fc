// rve_solve512.hip -- the batched RVE solver compiled with 512-thread
// workgroups (eight wave64) into namespace fehmm::nt512.  Used for 2D plans
// whose LDS fronts leave room for one workgroup per CU only: the same local
// memory then carries twice the waves (front slices of the wave phase, loads
// in flight, trailing-update tiles).
#define FEHMM_NT 512
#define FEHMM_VARIANT nt512
#include "rve_solve.hip"
