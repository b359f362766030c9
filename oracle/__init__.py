"""CPU oracle for the F2M gradient descent procedure (arXiv 2011.08170).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path
(the HIP library and its binding) never does.  It shares no code with the
HIP library.

`core` wraps the plain C oracle (GDP rule, certificate, exact optimum by
min-cost flow on the double cover); `exact` holds pure-Python checkers
(brute force over {0, 1/2, 1} edge vectors, exact-rational simplex) used to
pin the C oracle; `sec` is the GDP with subtour-elimination rows (F2M plus
rows x(delta(S)) >= 2 with multipliers >= 0, the extension of Sec. 5) in
plain numpy, pinned by `exact`'s rational LP with those rows.
"""
from . import core, exact, sec  # noqa: F401
