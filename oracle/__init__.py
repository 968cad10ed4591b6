"""CPU oracle for the Chebyshev / stencil-SpMMV path -- TEST INFRASTRUCTURE.

Plain, slow, obviously correct float64 / complex128 implementations written
from the paper (Pieper, Hager, Fehske, "A domain-specific language and
matrix-free stencil code for investigating electronic properties of Dirac and
topological materials", arXiv:1708.09689).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The product
(``paper_1708_09689_amd``) never imports it and shares no code with it; the
only common dependency is the seeded input generator module ``workloads``.

Modules
-------
lattice      cuboid indexing and per-dimension periodic/open neighbours (Sec. 3.4)
models       Hamiltonians as lists of hopping terms, from the model equations
             of Sec. 2 (graphene 4-site cell, graphene 2-site cell,
             3D topological insulator, Weyl semimetal)
hamiltonian  explicit sparse H assembled from those terms (the plain
             definition the matrix-free stencil must reproduce)
spmmv        y = alpha (H x - beta x) + gamma z per column, and the partial
             dot products of the fused kernel (Sec. 3.2, generated-code listing)
kpm          Chebyshev moments (direct and via the product doubling), Jackson
             kernel, DOS (Sec. 2.2 DOS equation, Sec. 4)
chebtp       Bessel J_k by Miller's backward recurrence, Chebyshev time
             propagation (Sec. 4.1, Eq. U_1)
chebfd       Chebyshev filter diagonalisation with Rayleigh-Ritz (Sec. 4.2)
spectral     momentum-resolved spectral function A(k, E) from Bloch start
             vectors (Sec. 2.2, Eq. ak)
rng          counter-based (SplitMix64) on-the-fly disorder field (Sec. 3.3)
adjoint      discrete adjoints of the KPM moments and of the Chebyshev time
             propagation with respect to the on-site potential, and central
             finite differences
omp_sweep    the Chebyshev step and the KPM moments over the explicit matrix
             in C++ with OpenMP (omp/cheb_omp.cpp), for the host's cores
"""
