"""CPU oracle for the round-off DCT approximation (Cintra & Bayer, arXiv 1402.6034).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the bench's
CPU-baseline leg may import this package.  The product path (the HIP library and
its Python binding) never imports, calls or links anything here, and this package
imports nothing from the product path: the two share no code, tables or helpers.

Everything is plain numpy: int64 for the integer transform, float64 otherwise.
Each function states the passage of the paper it follows.  Points where the paper
is silent are resolved by the readings listed in the module docstrings.

Parity status of each function (what pins it) is stated in its docstring; the
only unpinned part is the paper's own PSNR/UQI/MSE curves (its figures are not in
the text and its image set is not available).
"""
from .rdct import *  # noqa: F401,F403
from .image import *  # noqa: F401,F403
from .spectral import *  # noqa: F401,F403
from .quality import *  # noqa: F401,F403
from .codec import *  # noqa: F401,F403
