"""Plain FP64 CPU oracle for the semi-Lagrangian Newton--Krylov registration path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library under
``paper_1604_02153_amd/`` and its Python binding) imports, links or calls this
package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it, to check and to time the GPU path.

The oracle is written from Mang & Biros, "A semi-Lagrangian two-level
preconditioned Newton--Krylov solver for constrained diffeomorphic image
registration" (arXiv:1604.02153): the reduced-space formulation of section 3.1
(reduced gradient, eq. e:control-elim; GN Hessian matvec, eq. e:hessian-matvec),
the semi-Lagrangian transport of section 3.3.2 (eqs. e:state-slm .. e:inc-adj-slm,
characteristic e:characteristic), the preconditioners of section 3.4.2
(P_REG, eq. e:reg-precond; the nested two-level preconditioner) and the
Newton--Krylov loop of sections 3.4.1 and 3.5.  Every function is plain numpy
in float64; numpy's FFT and dense eigen-solver are the only library primitives.
"""

from .slnk_oracle import *  # noqa: F401,F403
from .slnk_oracle import __all__  # noqa: F401
