"""Independent FP64 CPU oracle for the 3-way ACA of Laplace-domain BEM tensors.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow reference written from the
paper (Haider, Rjasanow, Schanz, "Generalised adaptive cross approximation for
convolution quadrature based boundary element formulation"): the dense definition of
every frequency's single / double layer matrix (Sec. 3, spatial discretisation;
Laplace-domain kernel of Sec. 3, temporal discretisation) plus the 3D-ACA of Sec. 4
(Algorithm 1, eq. (norm), the dense-expansion pivot and the reordered product eq.
(product)).  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library
(``paper_2312_11219_amd``) and never imports it.

Parity status per function is listed in each module header.
"""
