"""CPU oracle for the 5D Shamir domain-wall fermion operator — TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 definitions written from the standard formulation of the
domain-wall Dirac operator that the paper names as its dominant kernel
(Introduction; Performance results, profiler figure of the main DWF kernel;
Conclusion, the node-local Wilson matrix).  The paper itself never writes the
operator down, so each convention is a stated reading (gamma basis, projector
pairing, boundary signs) listed with the functions below.

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package.  The HIP library never calls it and shares no code with it.

Modules:
  dwf_ref      numpy reference (operators, Schur form, CG, action, force)
  coracle      ctypes loader for the plain C/OpenMP oracle (liboracle_dwf.so)
"""
