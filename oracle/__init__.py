"""Plain FP64 CPU oracle for one time step of the two-phase Cahn-Hilliard
Navier-Stokes model (Khanwale et al., arXiv 2009.06628).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this
package: only the tests, the smoke check and the benchmark's CPU-baseline leg
use it.  It shares no code with the HIP library: it re-derives every operator
from its definition with numpy / scipy and solves every linear system exactly
(FFT / DCT diagonalisation or sparse direct factorisation), so any difference
from the GPU path is GPU arithmetic or solver error.

Continuous model: governing-equations section of the paper (momentum with the
Korteweg stress, thermodynamically consistent flux J, solenoidality, CH with
mu = psi' - Cn^2 lap phi), the double-well psi, the mixture maps rho, eta and
the pull-back phi* of the density / viscosity remark.  The paper's own time
and space discretisation (Crank-Nicolson + stabilised FEM + Newton) is not a
uniform-grid split step; the discrete algorithm implemented here is the
reading documented in the repository's design notes ("Algorithm S"):
first-order linear stabilised CH step, flux-form phi update, consistent mass
flux, skew-symmetric momentum advection, potential-form surface tension and a
variable-density pressure projection on a MAC grid.

Parity pins: every function is pinned by a CPU test under tests/ that checks
it against something other than itself (exact identities, closed forms,
invariants, brute force on tiny inputs).  Functions without such a pin say
"parity unpinned" in their docstring.
"""
from .grid import MACGrid  # noqa: F401
from .chns import (  # noqa: F401
    Params, coefficients, step, run, diagnostics, ch_operator_symbol,
)
