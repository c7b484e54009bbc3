"""Plain FP64 CPU oracle of the FFT strain-gradient crystal-plasticity method.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the GPU library never does, and the two share no
code.  Everything here is written for clarity, not speed: numpy arrays, numpy's FFT
as the discrete Fourier transform, dense per-voxel linear algebra, finite-difference
tangents.

Modules
  tables        FCC slip systems, interaction matrix, dislocation-segment matrix (Sec. 2.1)
  elasticity    cubic stiffness, rotations, slip-plane shear modulus (Table 2)
  spectral      rotated-scheme frequencies, projection operator, spectral curl (App. A, B)
  constitutive  finite-strain SGCP material point (eqs. 1-9, 14)
  solver        Galerkin-FFT Newton / conjugate-gradient homogenization (eqs. 15-18)
  nye           Nye tensor and minimum-norm GND densities (eqs. 10-13, App. B), and the
                transpose of that chain (adjoint form)
  reference     independent reference solutions used to pin the above
                (material point, laminate, dense Galerkin solve)

Voxel arrays are shaped (nz, ny, nx, ...) so that the flat index has x fastest;
spatial direction d (x=0, y=1, z=2) is array axis 2 - d.
"""
