"""The oracle's pins catch plausible mistakes (CPU only).

Each case copies the oracle's C source, plants one mistake by a textual
substitution, compiles the copy into a temporary directory and checks that
at least one pin fails against it (and that the same pins pass against the
unmodified oracle, which the pin tests themselves establish). Nothing here
touches the GPU library.
"""
import pytest

import oracle
from tests import test_oracle_pins as P

# (name, text in cloak_oracle.c, replacement, pins that must catch it)
MUTATIONS = [
    ("bottom cap normal points into the cloak",
     "if (surf == SURF_BOTTOM || surf == EV_BOTTOM) { n[0] = 0; n[1] = 0; n[2] = -1; return; }",
     "if (surf == SURF_BOTTOM || surf == EV_BOTTOM) { n[0] = 0; n[1] = 0; n[2] = 1; return; }",
     (P.test_finite_radial_ordinary_caps_closed_form, P.test_finite_azimuthal_extraordinary_caps_closed_form)),
    ("total internal reflection about the radial normal on every surface",
     "        w *= Rref[branch];\n        reflect(y + 3, nn);",
     "        w *= Rref[branch];\n        outward_normal(SURF_SIDE, y, nn);\n        reflect(y + 3, nn);",
     (P.test_finite_radial_ordinary_caps_closed_form, P.test_finite_azimuthal_extraordinary_caps_closed_form)),
    ("entry through the top cap accepted only over the metal disk's radius",
     "        if (s > 0.0 && x * x + y * y <= c->b * c->b && s < best) {\n            best = s; *surf = SURF_TOP;",
     "        if (s > 0.0 && x * x + y * y <= c->a * c->a && s < best) {\n            best = s; *surf = SURF_TOP;",
     (P.test_finite_radial_ordinary_caps_closed_form, P.test_finite_azimuthal_extraordinary_caps_closed_form)),
    ("Hamiltonian drift not checked at outer interfaces",
     "if (!(fabs(hamiltonian(c, branch, y) - 1.0) <= 1e-3)) { status = ORC_DIVERGED; break; }",
     "",
     (P.test_diverged_rule_at_outer_interfaces,)),
]


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(name, old, new, pins, tmp_path):
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    path = oracle.build_variant(src.replace(old, new), str(tmp_path))
    caught = []
    with oracle.use_library(path):
        for pin in pins:
            try:
                pin()
            except AssertionError:
                caught.append(pin.__name__)
    assert caught, f"no pin caught: {name}"
