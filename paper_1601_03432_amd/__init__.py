"""libsmpm: deflated Schur complement solver for the SMPM Poisson-Neumann
problem on AMD MI355X (gfx950).  See include/smpm.h for the C ABI; the Python
binding is paper_1601_03432_amd.smpm."""
