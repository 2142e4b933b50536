"""CPU oracle (test infrastructure only; the product never imports it)."""
from .knng_oracle import *  # noqa: F401,F403
