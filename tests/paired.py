"""The oracle in both of its forms, stepped side by side (test infrastructure).

GPU parity tests compare the library against the deviation form at the tight
FP64 bars (1e-12) and against the literal form -- the populations f_i as the
paper's equations write them, with plain sums -- at bars that add the literal
form's own rounding, measured in tests/test_oracle_forms.py:
  velocity    max|du| <= tol_u * max|u| + 2e-15
  density     max|drho| <= max(tol_rho, 5e-13)
  populations max|df| <= max(tol_f, 2e-13)
  force       max|dF| <= tol_F * F_scale + 1e-15 n, with tol_F >= 1e-11 and n the
              number of force terms (boundary links, or Lagrangian points)
The literal form's Eq. 17 sum adds one term per link, each carrying the
populations' own rounding (~1e-16 relative on values up to ~0.4), so its
absolute floor grows with the number of links.
"""
from oracle import Oracle

LITERAL_FLOOR = {"u": 2e-15, "rho": 5e-13, "f": 2e-13, "F_rel": 1e-11, "F_abs_per_term": 1e-15}


def force_terms(orc):
    """Terms of the force sums: boundary links, else Lagrangian points."""
    return max(len(orc.links()["cell"]), getattr(orc, "nlag", 0), 1)


_MUTATORS = {"set_solids", "set_lagrangian", "set_ibm_iters", "set_ibm_delta", "set_ibm_inner", "step", "set_f",
             "set_h", "set_free", "set_threads", "set_boundaries", "set_cover"}


class PairedOracle:
    """Forwards every call that changes the state to both forms; queries
    answer from the deviation form; ``lit`` is the literal one."""

    def __init__(self, *args, threads=1, **kw):
        kw.pop("form", None)
        self.dev = Oracle(*args, form="h", threads=threads, **kw)
        self.lit = Oracle(*args, form="f", threads=threads, **kw)

    def __getattr__(self, name):
        attr = getattr(self.dev, name)
        if name in _MUTATORS:
            def both(*a, **k):
                getattr(self.lit, name)(*a, **k)
                return attr(*a, **k)
            return both
        return attr
