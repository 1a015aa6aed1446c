"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only *defines problems*: the small direction matrices A_mu of a
Kronecker-sum operator K = A_d (+) ... (+) A_1 (paper section 1, eq. kronsum),
initial data, the name and parameters of the nonlinearity g, the step size,
the scheme name and the step count.  It holds none of the method's
arithmetic (no phi-functions, no mode products, no time stepping), so both
the CPU oracle and the GPU path can consume exactly the same arrays.

Layout convention: a tensor U of size n_1 x ... x n_d is held in natural
index order ``U[i_1, ..., i_d]`` (numpy shape ``(n_1, ..., n_d)``).  The
paper's vec() stacks columns, i.e. the first index runs fastest; device
memory uses that order, which is the C-contiguous array ``U.T`` of shape
``(n_d, ..., n_1)``.  ``to_memory_order`` / ``from_memory_order`` convert.
"""

from .problems import (  # noqa: F401
    Problem,
    RiccatiInstance,
    allen_cahn_2d,
    adr_3d,
    nls_3d,
    diffusion_reaction_3d,
    riccati_batch,
    adr_paper,
    random_dense_problem,
    dirichlet_d2,
    dirichlet_d1,
    periodic_d2,
    to_memory_order,
    from_memory_order,
    SCHEMES,
    NONLINEARITIES,
)
