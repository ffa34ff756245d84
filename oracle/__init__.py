"""FP64 CPU oracle for the hyperbolic self-gravity hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.  The
HIP library never does, and this package never imports the HIP library: the two
share no code.  The only module both sides use is ``workloads`` (seeded input
generators, none of the method's arithmetic).

What each part follows (paper: Hirai, Nagakura, Okawa & Fujisawa,
arXiv:1602.05700), and what pins it (tests/test_oracle_pins.py):

* ``hgs_oracle.c: orc_substeps`` -- explicit leapfrog of the inhomogeneous wave
  equation, Eq. (2), rho frozen over the sub-cycled steps (Sec. 2).  Optional
  damping eta (an extension, eta = 0 is Eq. (2)).  Pinned by: the closed-form
  amplitude of a single Dirichlet eigenmode (eta = 0 and eta > 0), the
  stability limit c dt/dx = 1/sqrt(3), the discrete Poisson solution (DST-I and
  dense LU) being a fixed point, exact conservation of the discrete energy at
  eta = 0, exactness on quadratic potentials, linearity in rho.
* ``orc_moments`` / ``orc_boundary`` -- Dirichlet outer boundary from a
  multipole expansion of rho (Sec. 2 and Sec. 4, Table I footnote c).  Pinned
  by: the Legendre addition theorem evaluated by brute force over cells,
  scipy's spherical harmonics, the monopole -G M / r, and convergence toward
  the free-space direct sum as lmax grows.
* ``orc_laplacian`` / ``orc_residual`` -- the steady state Eq. (1) in discrete
  form.  Pinned by: the discrete Gauss law (telescoping flux), R_b = 1 at a
  zero state, the DST-I solution giving round-off residuals, second-order
  convergence toward the closed-form Gaussian potential.
* ``orc_substeps_local`` / ``orc_local_ghosts`` / ``orc_residual_local`` --
  local outer boundaries whose ghosts follow the interior every substep: the
  Robin condition the paper uses by default (a monopole far field, Sec. 4)
  read as r_g phi_g = r_i phi_i; its radiative form
  d(r phi)/dt + c d(r phi)/dr = 0 (box scheme); periodic with the domain-mean
  density subtracted from the source (Sec. 4).  Pinned by
  (tests/test_oracle_bc.py): exactness on -G M / r, a sparse direct solve of
  the Robin linear system (steady state of both Robin and outgoing), an FFT
  solve with the 7-point symbol (periodic), a free pulse leaving through the
  outgoing boundary but not through zero-Dirichlet or static Robin ones, and
  relaxation of a zero start without damping through the outgoing boundary.
* ``orc_gradient`` -- g = -grad phi by central differences (the paper is silent
  on the discretisation).  Pinned by exactness on quadratics and second-order
  convergence on the Gaussian.
* ``poisson.py`` -- discrete Dirichlet Poisson solve by DST-I, the limit the
  method converges to (Eq. (1)); pinned by a dense LU solve on small grids.
  ``mean_relative_error`` is the paper's average relative error against the
  Poisson solution (Sec. 4, Eqs. (5)-(6)), pinned by closed forms (uniform and
  alternating relative offsets).
* ``analytic.py`` -- closed forms (uniform sphere, Gaussian, cube self
  potential) and brute-force sums used as pins.
* ``nn.py`` -- FP64 3D convolution network pieces (forward and backward) for the
  learned warm start; pinned by central finite differences.
* ``nested.py`` -- a coarse outer level of twice the cell size around the grid
  (Sec. 4 names nested grids as a way to move the boundary out): 2x2x2 means
  as the coarse source, trilinear interpolation of the coarse potential at the
  fine ghost centres.  Pinned by (tests/test_oracle_nested.py): exactness of
  the interpolation on affine fields, mass conservation of the source, the
  damped iteration reaching the composite steady state of a sparse Robin solve
  and DST-I solves (two and three levels), and the error against the
  free-space potential falling as the coarse level extends further.

The boundary study of Sec. 4 (Table I, kept as tests/golden/table1_models.txt)
pins the outer boundaries together: at the table's domain ratios around one
hydro grid the Robin boundary's error falls as the domain widens, and the
multipole Dirichlet boundary on the hydro grid lies between the smallest and
the widest Robin domain, the order the paper reports
(tests/test_oracle_table1.py).

Parity unpinned: no potential value of the paper's can be compared, because
the paper prints no worked example, table of potentials or figure data (all
figures are placeholders in the source text).
"""
from .core import Grid, Oracle, lib  # noqa: F401
