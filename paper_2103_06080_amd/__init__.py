"""MI355X-native exponential-integrator/WENO5 step for the KZK-type sonic-boom equation."""
