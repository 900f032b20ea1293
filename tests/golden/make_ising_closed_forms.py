"""Writes ``ising_closed_forms.json``: exact 2D Ising values at beta = 0.3, 0.4, 0.5.

Closed forms (square lattice, J = 1, two bonds per site):

* free energy (Onsager 1944): ``-beta f = ln(2 cosh 2b) + (1/pi) int_0^{pi/2}
  ln[(1 + sqrt(1 - k^2 sin^2 t)) / 2] dt`` with ``k = 2 sinh 2b / cosh^2 2b``;
* nearest-neighbour correlation ``<s s> = (1/2) d(-beta f)/d beta``
  ``= (1/2) coth 2b [1 + (2/pi)(2 tanh^2 2b - 1) K(k)]``;
* spontaneous magnetisation (Yang 1952): ``m = (1 - sinh^-4 2b)^{1/8}`` for
  ``b > b_c = ln(1 + sqrt 2) / 2``, else 0;
* nearest diagonal correlation ``<s(0,0) s(1,1)>`` (McCoy & Wu, The
  Two-Dimensional Ising Model, 1973): ``(2/pi) E(k)`` with
  ``k = sinh^-2 2b`` for ``b > b_c``, and ``(2/(pi k)) [E(k) - (1 - k^2) K(k)]``
  with ``k = sinh^2 2b`` for ``b < b_c`` (K, E complete elliptic integrals of
  modulus k); both give 2/pi at b_c, ``1 - 4 e^{-8b}`` at low and ``2 b^2``
  at high temperature, the leading terms of the series in those limits.

Computed with mpmath at 40 digits; nothing here calls the oracle.
Run: ``python tests/golden/make_ising_closed_forms.py``.
"""
import json
import os

import mpmath as mp

mp.mp.dps = 40


def closed_forms(b):
    b = mp.mpf(b)
    k = 2 * mp.sinh(2 * b) / mp.cosh(2 * b) ** 2
    integral = mp.quad(lambda t: mp.log((1 + mp.sqrt(1 - k ** 2 * mp.sin(t) ** 2)) / 2),
                       [0, mp.pi / 2])
    mbf = mp.log(2 * mp.cosh(2 * b)) + integral / mp.pi
    ss = mp.coth(2 * b) / 2 * (1 + 2 / mp.pi * (2 * mp.tanh(2 * b) ** 2 - 1)
                               * mp.ellipk(k ** 2))
    bc = mp.log(1 + mp.sqrt(2)) / 2
    m = (1 - mp.sinh(2 * b) ** -4) ** (mp.mpf(1) / 8) if b > bc else mp.mpf(0)
    if b > bc:
        kd = 1 / mp.sinh(2 * b) ** 2
        diag = 2 / mp.pi * mp.ellipe(kd ** 2)
    else:
        kd = mp.sinh(2 * b) ** 2
        diag = 2 / (mp.pi * kd) * (mp.ellipe(kd ** 2) - (1 - kd ** 2) * mp.ellipk(kd ** 2))
    return {"minus_beta_f": mp.nstr(mbf, 25), "nn_correlation": mp.nstr(ss, 25),
            "magnetisation": mp.nstr(m, 25), "diag_correlation": mp.nstr(diag, 25)}


if __name__ == "__main__":
    out = {"source": "Onsager 1944 (free energy), its beta-derivative (bond "
                     "correlation), Yang 1952 (magnetisation), McCoy & Wu 1973 "
                     "(diagonal correlation); mpmath, 40 digits",
           "values": {str(b): closed_forms(b) for b in (0.3, 0.4, 0.5)}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ising_closed_forms.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
