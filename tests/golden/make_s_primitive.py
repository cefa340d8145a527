"""Writes s_primitive_closed_form.txt from the closed form of one normalised
s Gaussian (AO equations for chi and g with n = (0,0,0), one primitive):
chi = (2g/pi)^(3/4) exp(-g r^2), d chi/dx = -2 g x chi,
lap chi = (4 g^2 r^2 - 6 g) chi.  Uses only the math module."""
import math
import os

rows = []
for g in (0.15, 1.0, 7.5):
    for (x, y, z) in ((0.3, -0.2, 0.1), (1.1, 0.4, -0.7), (-0.05, 0.02, 0.9)):
        r2 = x * x + y * y + z * z
        chi = (2 * g / math.pi) ** 0.75 * math.exp(-g * r2)
        rows.append((g, x, y, z, chi, -2 * g * x * chi, (4 * g * g * r2 - 6 * g) * chi))
with open(os.path.join(os.path.dirname(__file__), "s_primitive_closed_form.txt"), "w") as f:
    f.write("# gamma x y z chi dchi/dx lap_chi  (closed form, one normalised s primitive at the origin)\n")
    for r in rows:
        f.write(" ".join(repr(v) for v in r) + "\n")
