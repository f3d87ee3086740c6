"""MI355X-native space-time multigrid smoothing step for (p,delta)-Navier-Stokes."""
